// C ABI of libpwdf (declarations and contract: include/pwdf.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/pwdf.h"
#include "kernel_common.h"
#include "kernels.h"
#include "plan.h"

using namespace pwdf;

// Per-launch HIP-event timing (diagnostic mode, off by default).
struct ProfRec {
  int id;
  hipEvent_t a, b;
  double units;
};
struct ProfAgg {
  int64_t launches = 0;
  double ms = 0.0, units = 0.0;
};

// Launch-shape choice: segment length, per class L multipliers of the default
// wave targets of the rho and J passes (chunk counts follow from them), and
// whether independent launches of one pass fan out over the internal streams
// (fork = 1) or follow each other on the caller's stream (fork = 0).
struct Tune {
  int seg_len = 8;
  double mrho[kMaxLsum + 1];
  double mj[kMaxLsum + 1];
  int fork = 1;
  // FP32-MFMA form: measured milliseconds of the per-class launches (rho tail,
  // rho head, J tail, J head) and whether the passes order their launches by
  // them (see class_schedule)
  double cost[4][kMaxLsum + 1];
  int lpt = 0;
  Tune() {
    for (int L = 0; L <= kMaxLsum; ++L) {
      mrho[L] = mj[L] = 1.0;
      for (int i = 0; i < 4; ++i) cost[i][L] = 0.0;
    }
  }
};

constexpr int kAux = 4;  // internal streams for independent per-class launches

struct GraphCache {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int ndm = 0;
  const void *Dk = nullptr;
  void *Jk = nullptr, *EJ = nullptr;
};

struct pwdf_ctx {
  Plan plan;
  PlanInput in;
  Tune tune;
  bool prof_on = false;
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> prof_pool;
  size_t prof_next = 0;
  std::vector<std::string> prof_names;
  std::vector<ProfAgg> prof_agg;
  Dev dev;
  std::vector<void *> owned;  // device allocations of the current setup
  double *Escr = nullptr;     // [max_ndm] energies of diagnostic calls
  double *ERpart = nullptr;   // [max_ndm][256] partials of the real-space energy
  int blocks_ndm = 0;         // densities whose D(L) / J(L) blocks the workspace holds
  bool ready = false;         // the device setup is complete (false after a failed one)
  hipStream_t aux[kAux] = {};
  hipStream_t cap = nullptr;  // capture / tuning stream
  hipEvent_t ev_fork = nullptr, ev_join[kAux] = {};
  GraphCache gc;
  std::string err;
  int device = 0;
  int max_ndm = 1;
  pwdf_precision prec = PWDF_FP64;
  int jk_layout = PWDF_JK_FULL;
  int dk_layout = PWDF_DK_FULL;
};

namespace {

thread_local std::string g_create_err;

pwdf_status fail(pwdf_ctx *c, pwdf_status s, const std::string &m) {
  if (c)
    c->err = m;
  else
    g_create_err = m;
  return s;
}

// build_plan marks parameters it cannot handle (as opposed to invalid ones)
pwdf_status plan_status(const std::string &why) {
  return why.rfind("unsupported:", 0) == 0 ? PWDF_EUNSUPPORTED : PWDF_EINVAL;
}

pwdf_status hip_fail(pwdf_ctx *c, hipError_t e, const char *where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(c, e == hipErrorOutOfMemory ? PWDF_ENOMEM : PWDF_EDEVICE, m);
}

// Every device allocation of the library goes through dev_malloc / dev_free:
// g_live counts the allocations held (all contexts), g_alloc_budget >= 0 makes
// every allocation after that many more fail (pwdf_debug_fail_alloc).
std::atomic<int64_t> g_live{0};
std::atomic<int> g_alloc_budget{-1};

hipError_t dev_malloc(void **p, size_t n) {
  int b = g_alloc_budget.load();
  while (b >= 0) {
    if (b == 0) return hipErrorOutOfMemory;
    if (g_alloc_budget.compare_exchange_weak(b, b - 1)) break;
  }
  const hipError_t e = hipMalloc(p, n);
  if (e == hipSuccess) ++g_live;
  return e;
}

void dev_free(void *p) {
  if (p && hipFree(p) == hipSuccess) --g_live;
}

template <class T>
hipError_t upload(pwdf_ctx *c, const std::vector<T> &v, const T **out) {
  void *p = nullptr;
  size_t n = std::max<size_t>(1, v.size()) * sizeof(T);
  hipError_t e = dev_malloc(&p, n);
  if (e != hipSuccess) return e;
  c->owned.push_back(p);
  if (!v.empty()) {
    e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
  }
  *out = (const T *)p;
  return hipSuccess;
}

template <class T>
hipError_t alloc(pwdf_ctx *c, size_t count, T **out) {
  void *p = nullptr;
  hipError_t e = dev_malloc(&p, std::max<size_t>(1, count) * sizeof(T));
  if (e != hipSuccess) return e;
  c->owned.push_back(p);
  *out = (T *)p;
  return hipSuccess;
}

void free_device(pwdf_ctx *c) {
  for (void *p : c->owned) dev_free(p);
  c->owned.clear();
}

void drop_graph(pwdf_ctx *c) {
  if (c->gc.exec) (void)hipGraphExecDestroy(c->gc.exec);
  if (c->gc.graph) (void)hipGraphDestroy(c->gc.graph);
  c->gc = GraphCache();
}

// Launch shapes: spread each pass over about 4096 waves so that every wave of
// every class does about the same work (the classes of one pass run
// concurrently).  rho: lane = segment, a class is split into pair chunks.
// J: lane = pair, a class is split into segment chunks; a wave costs the same
// whether or not all 64 pairs are present, so the J weights count padded lanes.
// Per pair and point the cost is about 2L + 10 operations plus the segment start
// (two exponentials, one sincos, the NT coefficients) spread over SEG points.
// In the FP64 rho pass each class group (L <= 2, L >= 3: its two launches) gets
// at least kMinGroupWaves of the waves: a group with little work, usually the
// high classes, would otherwise run as a few long waves, and that latency is its
// launch time whenever it does not overlap the other group.  (The J pass keeps
// the plain share: more high-class J chunks cost more in the back-transform,
// which sums them, than they save.)  A rho chunk holds at least 4 pairs (the 4
// waves of its blocks share them).
// The tune multipliers scale the chunk counts per class.
// columns of a partial row: slots (FP64 form), points of the tail (FP32-MFMA form)
// complex intermediates of the GPW transforms, per density
size_t gpw_a_size(const Dev &d) { return (size_t)d.gN[2] * d.gN[1] * (2 * d.gM[0] + 1); }
size_t gpw_b_size(const Dev &d) { return (size_t)d.gN[2] * (2 * d.gM[1] + 1) * (2 * d.gM[0] + 1); }
size_t gpw_c_size(const Dev &d) { return (size_t)(2 * d.gM[2] + 1) * (2 * d.gM[1] + 1) * (2 * d.gM[0] + 1); }

size_t part_cols(const Dev &d) { return d.fp32 ? (size_t)std::max(1, d.npts - d.npts_head) : (size_t)d.nslot; }

// Host-side work lists of the FP32-MFMA form (see Dev), uploaded by setup_device.
struct WorkLists {
  std::vector<int4> rho_items, j_items;
  std::vector<int> rows_of_block, jn_of, slot_pidx;
};

// FP64 form: segment chunks of both passes.  In the FP32-MFMA form these give
// the segment chunks of the gradient's FP64 force moments; its own passes are
// laid out by fp32_shapes.
void choose_shapes_fp64(const Plan &p, Dev &d, const Tune &tn, int max_ndm) {
  const int SEG = p.seg_len;
  const double target = 4096.0;
  // the low-L classes share S across d.ndb densities per block (at most 32 / SEG,
  // chosen at launch); chunk counts are those of one density block (a batch
  // adds blocks along the density axis of the grid)
  d.ndb = max_ndm >= 4 ? 4 : (max_ndm >= 2 ? 2 : 1);
  d.rho_bs = 256;  // 64 segments x 4 waves sharing them
  double wsumR = 0.0, wsumJ = 0.0, wR[kMaxLsum + 1], wJ[kMaxLsum + 1];
  for (int L = 0; L <= kMaxLsum; ++L) {
    const int np = p.L_p1[L] - p.L_p0[L];
    const double cost = 2.0 * L + 10.0 + (70.0 + nherm(L)) / SEG;
    wR[L] = np > 0 ? (double)np * cost : 0.0;
    wJ[L] = np > 0 ? (double)((np + 63) / 64) * 64.0 * cost : 0.0;
    wsumR += wR[L];
    wsumJ += wJ[L];
  }
  // rho: a chunk spans the G set in groups of 64 segments, four waves each; J:
  // the segments are split into chunks
  const int ngi = p.nseg();
  const int rho_waves_per_chunk = std::max(4, ((ngi + 63) / 64) * 4);
  wsumR = std::max(wsumR, 1.0);  // no pairs: every class is skipped below
  wsumJ = std::max(wsumJ, 1.0);
  constexpr double kMinGroupWaves = 1024.0;
  double gR[2] = {0.0, 0.0}, gJ[2] = {0.0, 0.0};
  for (int L = 0; L <= kMaxLsum; ++L) {
    gR[L > 2] += wR[L];
    gJ[L > 2] += wJ[L];
  }
  double tR[2], tJ[2];  // waves of each group
  for (int g = 0; g < 2; ++g) {
    tR[g] = std::max(target * gR[g] / wsumR, kMinGroupWaves);
    tJ[g] = target * gJ[g] / wsumJ;
    gR[g] = std::max(gR[g], 1.0);
    gJ[g] = std::max(gJ[g], 1.0);
  }
  int rows = 0;
  int64_t yoff = 0;
  for (int L = 0; L <= kMaxLsum; ++L) {
    int np = p.L_p1[L] - p.L_p0[L];
    d.rho_row0[L] = rows;
    d.yhat_off[L] = yoff;
    if (np <= 0) {
      d.rho_chunks[L] = 0;
      d.rho_ppc[L] = 1;
      d.j_chunks[L] = 0;
      d.j_spc[L] = 1;
      continue;
    }
    int ch = (int)std::lround(tR[L > 2] * (wR[L] / gR[L > 2]) * tn.mrho[L] / rho_waves_per_chunk);
    ch = std::max(1, std::min((np + 3) / 4, ch));
    int ppc = (np + ch - 1) / ch;
    ch = (np + ppc - 1) / ppc;
    d.rho_chunks[L] = ch;
    d.rho_ppc[L] = ppc;
    rows += ch;
    const int jw = (np + 63) / 64;  // waves per chunk: a pair per lane
    int jc = (int)std::lround(tJ[L > 2] * (wJ[L] / gJ[L > 2]) * tn.mj[L] / jw);
    jc = std::max(1, std::min(ngi, jc));
    int spc = std::max(1, (ngi + jc - 1) / jc);
    jc = (ngi + spc - 1) / spc;  // 0 when the G set is empty
    d.j_chunks[L] = jc;
    d.j_spc[L] = spc;
    yoff += (int64_t)jc * nherm(L) * np;
  }
  // force moments of degree L+1 over the class-L pairs, same segment chunks as J
  int64_t foff = 0;
  for (int L = 0; L <= kMaxLsum; ++L) {
    int np = p.L_p1[L] - p.L_p0[L];
    d.yF_off[L] = foff;
    if (np > 0 && L < kMaxLsum) foff += (int64_t)d.j_chunks[L] * nherm(L + 1) * np;
  }
  d.yF_size = std::max<int64_t>(1, foff);
  d.nrows = std::max(1, rows);
  d.ngroups = std::min(d.nrows, 64);
  d.rows_per_group = (d.nrows + d.ngroups - 1) / d.ngroups;
  d.ngroups = (d.nrows + d.rows_per_group - 1) / d.rows_per_group;
  d.yhat_size = std::max<int64_t>(1, yoff);
  d.nred_blocks = (p.nslot() + 3) / 4;
}

// FP32-MFMA form: work items of both passes over the tail of the G set and the
// chunks of the head (see Dev).  Both passes aim at about kItemWaves waves in
// items of equal cost: per K-step of a wave (4 pairs or points) the pair factor
// S costs ~120 cycles per group of N-tiles and each N-tile two MFMAs of 32
// cycles; rho runs a class's ceil(nt / 8) groups one after the other in one item,
// J one group per workgroup (grid z).  A run of FP32 accumulation covers at most
// kMaxFp32Run pairs or points (the head, where the largest terms are, is in
// FP64).  The tune multipliers scale the item counts per class.
void fp32_shapes(const Plan &p, Dev &d, const Tune &tn, WorkLists &wl) {
  constexpr double kItemWaves = 8192.0;
  constexpr int kMaxFp32Run = 1024, kMinRun = 16;
  constexpr int kHeadWaves = 2048, kHeadMinPairs = 32;
  constexpr int kHeadJBlocks = 512, kHeadJMinPts = 32;
  constexpr int kRhoZWaves = 2048;  // tail rho: spread a class's N-tile groups below this many waves
  const int nh = d.npts_head, npts = (int)p.pts.size(), ntail = npts - nh;
  const int nb = (ntail + 63) / 64;
  std::vector<double> tg2(ntail);
  for (int i = 0; i < ntail; ++i) tg2[i] = p.pts[nh + i].g2;
  wl = WorkLists();
  wl.slot_pidx.assign(p.nslot(), -1);
  for (int i = 0; i < npts; ++i) wl.slot_pidx[p.pts[i].slot] = i;
  // per class: active pairs of each point block (cut order: gc2 descending) and
  // active points of each pair block (points: |G|^2 ascending)
  std::vector<std::vector<int>> nact(kMaxLsum + 1), nactp(kMaxLsum + 1);
  double WR = 0.0, WJ = 0.0, costR[kMaxLsum + 1], costJ[kMaxLsum + 1];
  int ngr[kMaxLsum + 1];
  for (int L = 0; L <= kMaxLsum; ++L) {
    const int np = p.L_p1[L] - p.L_p0[L];
    const int nt = std::max(1, d.ncols32[L] / 16);
    ngr[L] = tile_groups(nt);
    const int ntg = group_tiles(nt);
    costR[L] = ngr[L] * (120.0 + 64.0 * ntg);
    costJ[L] = 120.0 + 64.0 * ntg;
    if (np <= 0) continue;
    nact[L].resize(nb);
    for (int b = 0; b < nb; ++b) {
      const double g = tg2[64 * b];
      // first pair (cut order) whose cut lies below the block's shortest G
      int lo = 0, hi = np;
      while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (p.hot_cut[p.L_p0[L] + mid].gc2 >= g) lo = mid + 1; else hi = mid;
      }
      nact[L][b] = lo;
      WR += (lo / 4.0) * costR[L];
    }
    const int npb = (np + 63) / 64;
    nactp[L].resize(npb);
    for (int B = 0; B < npb; ++B) {
      const double c = p.hot_cut[p.L_p0[L] + 64 * B].gc2;
      nactp[L][B] = (int)(std::upper_bound(tg2.begin(), tg2.end(), c) - tg2.begin());
      WJ += ngr[L] * (nactp[L][B] / 4.0) * costJ[L];
    }
  }
  // item cost (cycles of one wave) for about kItemWaves waves, 4 per item
  const double CR = std::max(1.0, WR / (kItemWaves / 4.0)), CJ = std::max(1.0, WJ / (kItemWaves / 4.0));
  auto run_len = [&](double C, double cost, double mult, int cap) {
    int r = (int)std::lround(4.0 * C / cost / std::max(mult, 1e-3));
    r = std::max(kMinRun, std::min(cap, r));
    return (r + 3) / 4 * 4;
  };
  wl.rows_of_block.assign(std::max(1, nb), 0);
  wl.jn_of.assign(p.hot.size(), 0);
  int rows_h = 0;
  int64_t yoff = 0;
  for (int L = 0; L <= kMaxLsum; ++L) {
    const int np = p.L_p1[L] - p.L_p0[L];
    d.rho_item0[L] = (int)wl.rho_items.size();
    d.j_item0[L] = (int)wl.j_items.size();
    d.rho_nitems[L] = d.j_nitems[L] = 0;
    d.rho_h_row0[L] = rows_h;
    d.rho_h_chunks[L] = 0;
    d.rho_h_ppc[L] = 1;
    d.yhat_off[L] = yoff;
    d.jh_chunks[L] = 0;
    d.jh_ppc[L] = 1;
    if (np <= 0) continue;
    // J over the head (FP64 MFMA): split over the head points into yhat chunks
    // [0, hc) so that a class of few pairs still fills about kHeadJBlocks
    // workgroups (each chunk at least kHeadJMinPts points)
    int hc = 0;
    if (nh > 0) {
      const int blocks = ((np + 63) / 64) * ngr[L];
      hc = std::max(1, std::min((kHeadJBlocks + blocks - 1) / blocks, (nh + kHeadJMinPts - 1) / kHeadJMinPts));
      d.jh_ppc[L] = (nh + hc - 1) / hc;
      hc = (nh + d.jh_ppc[L] - 1) / d.jh_ppc[L];
      d.jh_chunks[L] = hc;
    }
    // rho over the tail; a class of few items (the high classes, whose items walk
    // many N-tile groups) spreads its groups over grid z in slices, each slice
    // adding into a partial row of its own
    const int ppc = run_len(CR, costR[L], tn.mrho[L], kMaxFp32Run);
    int nit = 0;
    for (int b = 0; b < nb; ++b) nit += (nact[L][b] + ppc - 1) / ppc;
    int gps = ngr[L];
    if (nit > 0 && 4 * nit < kRhoZWaves) {
      const int want = std::min(ngr[L], (kRhoZWaves + 4 * nit - 1) / (4 * nit));
      gps = (ngr[L] + want - 1) / want;
    }
    const int zs = (ngr[L] + gps - 1) / gps;  // every slice holds at least one group
    d.rho_gps[L] = gps;
    d.rho_zs[L] = zs;
    for (int b = 0; b < nb; ++b)
      for (int q0 = 0; q0 < nact[L][b]; q0 += ppc) {
        wl.rho_items.push_back(make_int4(b, q0, std::min(nact[L][b], q0 + ppc), wl.rows_of_block[b]));
        wl.rows_of_block[b] += zs;
      }
    d.rho_nitems[L] = (int)wl.rho_items.size() - d.rho_item0[L];
    // J over the tail; a class of few pair blocks (the high classes) takes shorter
    // point runs, so that its launch still spreads over about kRhoZWaves waves
    // (more chunks of moments, which the back transform's chunk sum reads)
    int spc = run_len(CJ, costJ[L], tn.mj[L], kMaxFp32Run);
    {
      int nit = 0;
      for (int B = 0; B < (int)nactp[L].size(); ++B) nit += (nactp[L][B] + spc - 1) / spc;
      const int waves = 4 * nit * ngr[L];
      if (nit > 0 && waves < kRhoZWaves) {
        const int r = (int)((int64_t)spc * waves / kRhoZWaves);
        spc = std::max(kMinRun, (r + 3) / 4 * 4);
      }
    }
    int maxc = 0;
    for (int B = 0; B < (int)nactp[L].size(); ++B) {
      int c = 0;
      for (int s0 = 0; s0 < nactp[L][B]; s0 += spc, ++c)
        wl.j_items.push_back(make_int4(B, s0, std::min(nactp[L][B], s0 + spc), c));
      maxc = std::max(maxc, c);
      for (int r = 64 * B; r < std::min(np, 64 * B + 64); ++r) wl.jn_of[p.L_p0[L] + r] = hc + c;
    }
    d.j_nitems[L] = (int)wl.j_items.size() - d.j_item0[L];
    yoff += (int64_t)(hc + maxc) * nherm(L) * np;
    // the head (FP64 MFMA): rho in chunks of pairs x N-tile groups (one partial
    // row each), about kHeadWaves waves per class launch; J moments over all head
    // points in one chunk
    if (nh > 0) {
      const int waves_per_chunk = 4 * ((nh + 63) / 64) * ngr[L];
      const int want = std::max(1, kHeadWaves / waves_per_chunk);
      const int hp = std::max(kHeadMinPairs, (np + want - 1) / want);
      d.rho_h_ppc[L] = hp;
      d.rho_h_chunks[L] = (np + hp - 1) / hp;
      rows_h += d.rho_h_chunks[L] * ngr[L];
    }
  }
  int nrows = 1;
  for (int r : wl.rows_of_block) nrows = std::max(nrows, r);
  d.nrows = nrows;
  d.nrows_h = std::max(1, rows_h);
  // first reduction stage: up to 64 groups of the tail rows and of the head rows
  d.ngroups = std::min(std::max(d.nrows, nh > 0 ? d.nrows_h : 0), 64);
  d.rows_per_group = (d.nrows + d.ngroups - 1) / d.ngroups;
  d.rows_per_group_h = (d.nrows_h + d.ngroups - 1) / d.ngroups;
  d.yhat_size = std::max<int64_t>(1, yoff);
}

void choose_shapes(const Plan &p, Dev &d, const Tune &tn, int max_ndm, WorkLists &wl) {
  choose_shapes_fp64(p, d, tn, max_ndm);
  if (d.fp32) fp32_shapes(p, d, tn, wl);
}

// (Re)builds the device view of the plan: uploads and workspaces for the current
// segment length and tune.  Frees the previous setup first.
pwdf_status setup_device_impl(pwdf_ctx *c, const Tune &tn) {
  c->blocks_ndm = 0;
  drop_graph(c);
  free_device(c);
  c->tune = tn;
  Plan &p = c->plan;
  const PlanInput &in = c->in;
  Dev &d = c->dev;
  std::memset(&d, 0, sizeof(d));
  d.nk = p.nk;
  d.nbf = p.nbf;
  d.nshell = in.nshell;
  d.natm = in.natm;
  d.nseg = p.nseg();
  d.nslot = p.nslot();
  d.npts = (int)p.pts.size();
  d.seg_len = p.seg_len;
  d.nelem = p.nelem;
  d.vol = p.vol;
  for (int i = 0; i < 16; ++i) {
    d.cls_b0[i] = p.cls_b0[i];
    d.cls_b1[i] = p.cls_b1[i];
  }
  for (int L = 0; L <= kMaxLsum; ++L) {
    d.L_p0[L] = p.L_p0[L];
    d.L_p1[L] = p.L_p1[L];
    d.dhat_off[L] = p.dhat_off[L];
  }
  d.dhat_size = std::max<int64_t>(1, p.dhat_size);
  d.nsegJ = (int)p.sJ_code.size();
  d.nsegD = (int)p.sD_code.size();
  d.nsegDp = (int)p.sDp_code.size();
  for (int i = 0; i < 3; ++i) d.kmesh[i] = in.kmesh[i];
  d.nheavyJ = (int)p.heavyJ.size();
  d.nlightJ = (int)p.lightJ.size();
  d.jk_layout = c->jk_layout;
  d.dk_layout = c->dk_layout;
  d.pair_gcut = p.cut_on() ? 1 : 0;
  d.muu = p.M[p.ax[0]][p.ax[0]];
  d.fp32 = c->prec == PWDF_FP32_MFMA ? 1 : 0;
  d.npts_head = d.fp32 ? p.npts_head : 0;
  if (d.fp32) {
    d.ndmp = 1;
    while (d.ndmp < c->max_ndm) d.ndmp *= 2;
    int64_t off = 0;
    int lmax = 0;
    for (int L = 0; L <= kMaxLsum; ++L) {
      int npl = p.L_p1[L] - p.L_p0[L];
      d.ncols32[L] = ((nherm(L) * d.ndmp + 15) / 16) * 16;
      d.d32_off[L] = off;
      if (npl > 0) {
        off += (int64_t)npl * d.ncols32[L];
        lmax = L;
      }
    }
    d.ncolsW = d.ncols32[lmax];
    d.d32_size = off;
  }
  WorkLists wl;
  choose_shapes(p, d, tn, c->max_ndm, wl);

  hipError_t e;
#define UP(vec, field) \
  if ((e = upload(c, vec, &d.field)) != hipSuccess) return hip_fail(c, e, "uploading " #field);
  UP(p.segs, segs)
  UP(p.pts, pts)
  UP(p.valid_slots, valid_slots)
  d.nvalid = (int)p.valid_slots.size();
  UP(p.slot_v, slot_v)
  UP(p.hot, hot)
  UP(p.hot_rho, hot_rho)
  UP(p.rho_rank, rho_rank)
  UP(p.hot_cut, hot_cut)
  UP(p.cut_rank, cut_rank)
  UP(p.blk_cut, blk_cut)
  UP(p.aux, aux)
  UP(p.blocks, blocks)
  UP(p.elem_blk, elem_blk)
  UP(in.sh_l, sh_l)
  UP(in.sh_atom, sh_atom)
  UP(p.sp_off, sp_off)
  UP(p.sp_ent, sp_ent)
  UP(p.bf_shell, bf_shell)
  UP(p.bf_comp, bf_comp)
  UP(p.sJ_off, sJ_off)
  UP(p.sJ_code, sJ_code)
  UP(p.sJ_e0, sJ_e0)
  UP(p.eJ, eJ)
  UP(p.sD_el, sD_el)
  UP(p.heavyJ, heavyJ)
  UP(p.lightJ, lightJ)
  UP(p.sD_code, sD_code)
  UP(p.sD_e0, sD_e0)
  UP(p.eD, eD)
  UP(p.sDp_el, sDp_el)
  UP(p.sDp_code, sDp_code)
  UP(p.sDp_e0, sDp_e0)
  UP(p.eDp, eDp)
  UP(p.ttab, ttab)
  d.ndd = (int)p.dd_q.size();
  if (d.ndd > 0) {
    UP(p.dd_q, dd_q)
    UP(p.dd_L, dd_L)
    UP(p.dd_of, dd_of)
    UP(p.slot_vf, slot_vf)
  }
  if (d.ndd > 0) {
    // rho_D of the analytic route: about 2048 workgroups over (slot blocks x
    // chunks of DD pairs), at least 8 pairs per chunk
    const int bx = (d.nslot + 255) / 256;
    int nc = std::max(1, std::min((2048 + bx - 1) / bx, (d.ndd + 7) / 8));
    d.dd_ppc = (d.ndd + nc - 1) / nc;
    d.dd_chunks = (d.ndd + d.dd_ppc - 1) / d.dd_ppc;
  }
  d.gpw = (d.ndd > 0 && in.dd_gpw) ? 1 : 0;
  if (d.gpw) {
    for (int i = 0; i < 3; ++i) {
      d.gN[i] = p.gN[i];
      d.gM[i] = p.gM[i];
      d.gtiles[i] = p.gtiles[i];
    }
    d.gpts = (int64_t)p.gN[0] * p.gN[1] * p.gN[2];
    for (int c = 0; c < 3; ++c)
      for (int i = 0; i < 3; ++i) d.lat[c * 3 + i] = p.A[c][i];
    UP(p.dd_blk, dd_blk)
    UP(p.gP, gP)
    UP(p.gimg, gimg)
    UP(p.gimg_box, gimg_box)
    UP(p.gimg_off, gimg_off)
    UP(p.gtile_ent, gtile_ent)
    UP(p.gitem, gitem)
    UP(p.gitem_off, gitem_off)
    d.ngitems = (int)(p.gitem.size() / 3);
    UP(p.slot_miller, slot_miller)
  }
  if (d.fp32) {
    // n^k of every point: the products the epilogues formed on the device
    // (repeated multiplications, u then v then w; integers, exact while
    // |n|^(2 kMaxL) < 2^53)
    {
      constexpr Monos<2 * kMaxL> MT{};
      std::vector<double> pm(std::max<size_t>(1, p.pts.size() * (size_t)kMonoStride), 0.0);
      auto pw = [](double x, int e) {
        double r = 1.0;
        for (int i = 0; i < e; ++i) r *= x;
        return r;
      };
      for (size_t i = 0; i < p.pts.size(); ++i)
        for (int k = 0; k < kMonoStride; ++k)
          pm[i * kMonoStride + k] =
              pw(p.pts[i].nu, MT.u[k]) * pw(p.pts[i].nv, MT.v[k]) * pw(p.pts[i].nw, MT.w[k]);
      UP(pm, ptmono)
    }
    UP(wl.slot_pidx, slot_pidx)
    UP(wl.rho_items, rho_items)
    UP(wl.j_items, j_items)
    UP(wl.rows_of_block, rows_of_block)
    UP(wl.jn_of, jn_of)
  }
  {
    std::vector<double> st(kStartTab);
    start_tables(st.data());
    if ((e = upload(c, st, &d.start_tab)) != hipSuccess) return hip_fail(c, e, "uploading start tables");
  }
#undef UP
  {
    const double *ph;
    if ((e = upload(c, p.phD, &ph)) != hipSuccess) return hip_fail(c, e, "uploading phase tables");
    d.phD = (const double2 *)ph;
    if ((e = upload(c, p.phJ, &ph)) != hipSuccess) return hip_fail(c, e, "uploading phase tables");
    d.phJ = (const double2 *)ph;
    if ((e = upload(c, p.ptab, &ph)) != hipSuccess) return hip_fail(c, e, "uploading phase table");
    d.ptab = (const double2 *)ph;
    d.ptab_len = (int)(p.ptab.size() / 2);
  }
  const size_t M = (size_t)c->max_ndm;
#define AL(field, count) \
  if ((e = alloc(c, (count), &d.field)) != hipSuccess) return fail(c, PWDF_ENOMEM, "device allocation failed: " #field);
  AL(Dblk, M * p.nelem)
  AL(Jblk, M * p.nelem)
  // the FP32-MFMA form keeps the coefficients in the MFMA layout (d32_size per call)
  AL(dhat, d.fp32 ? (size_t)std::max<int64_t>(1, d.d32_size) : M * d.dhat_size)
  AL(yhat, M * d.yhat_size)
  AL(part, M * d.nrows * part_cols(d))
  AL(part2, M * d.ngroups * d.nslot)
  AL(rho, M * d.nslot)
  AL(Vc, M * d.nslot)
  AL(Epart, M * d.nred_blocks)
  if (d.ndd > 0) {
    AL(rhoD, M * d.nslot)
    AL(rhoDp, M * d.dd_chunks * d.nslot)
    AL(VDc, M * d.nslot)
    AL(ydd, M * d.ndd * kDDStride)
    AL(yddF, M * d.ndd * kDDStride)
  }
  if (d.gpw) {
    AL(grid_r, M * d.gpts)
    AL(grid_p, M * d.ngitems * 512)
    AL(grid_a, M * gpw_a_size(d))
    AL(grid_b, M * gpw_b_size(d))
    AL(grid_c, M * gpw_c_size(d))
    AL(gpw_part, M * d.ndd * kGpwEl)
  }
  AL(Jfold, M * (size_t)std::max(1, d.nsegJ))
  AL(yF, M * d.yF_size)
  d.nblocks = (int)p.blocks.size();
  AL(gblk, M * (size_t)d.nblocks * 6)
  if (d.npts_head > 0) AL(parth, M * d.nrows_h * d.npts_head)
  if (d.fp32) {
    AL(dh32, (size_t)std::max<int64_t>(1, d.d32_size))
    AL(wre, (size_t)d.nslot * d.ncolsW)
    AL(wim, (size_t)d.nslot * d.ncolsW)
    if (d.npts_head > 0) {
      AL(wre64, (size_t)d.npts_head * d.ncolsW)
      AL(wim64, (size_t)d.npts_head * d.ncolsW)
    }
    if ((e = hipMemset(d.dh32, 0, sizeof(float) * std::max<int64_t>(1, d.d32_size))) != hipSuccess)
      return hip_fail(c, e, "clearing operand buffer");
  }
#undef AL
  {
    // per atom: (block * 6 + 0) for shell a on the atom, (block * 6 + 3) for shell b
    std::vector<std::vector<int>> per(in.natm);
    for (int b = 0; b < d.nblocks; ++b) {
      per[in.sh_atom[p.blocks[b].sa]].push_back(b * 6);
      per[in.sh_atom[p.blocks[b].sb]].push_back(b * 6 + 3);
    }
    std::vector<int> off(in.natm + 1, 0), ent;
    for (int a = 0; a < in.natm; ++a) {
      off[a] = (int)ent.size();
      ent.insert(ent.end(), per[a].begin(), per[a].end());
    }
    off[in.natm] = (int)ent.size();
    if ((e = upload(c, off, &d.atom_off)) != hipSuccess || (e = upload(c, ent, &d.atom_ent)) != hipSuccess)
      return hip_fail(c, e, "uploading atom lists");
  }
  if ((e = alloc(c, M, &c->Escr)) != hipSuccess) return fail(c, PWDF_ENOMEM, "device allocation failed: energies");
  if ((e = alloc(c, M * 256, &c->ERpart)) != hipSuccess)
    return fail(c, PWDF_ENOMEM, "device allocation failed: energy partials");
  if ((e = alloc(c, 1, &d.nonfinite)) != hipSuccess) return fail(c, PWDF_ENOMEM, "device allocation failed: flag");
  if ((e = hipMemset(d.nonfinite, 0, sizeof(int))) != hipSuccess) return hip_fail(c, e, "clearing the input flag");
  return PWDF_OK;
}

// A failed setup releases what it had allocated and leaves the context unusable
// for device work (PWDF_ESTATE) until pwdf_destroy.
pwdf_status setup_device(pwdf_ctx *c, const Tune &tn) {
  c->ready = false;
  const pwdf_status s = setup_device_impl(c, tn);
  if (s != PWDF_OK) {
    free_device(c);
    std::memset(&c->dev, 0, sizeof(c->dev));
    c->Escr = c->ERpart = nullptr;
    return s;
  }
  c->ready = true;
  return PWDF_OK;
}

pwdf_status not_ready(pwdf_ctx *c) {
  return fail(c, PWDF_ESTATE,
              "the context's device setup failed (" + c->err + "); it takes no further device work: destroy it");
}

pwdf_status validate_ndm(pwdf_ctx *c, int ndm) {
  if (!c->ready) return not_ready(c);
  if (ndm < 1) return fail(c, PWDF_EINVAL, "ndm must be >= 1");
  if (ndm > c->max_ndm) return fail(c, PWDF_EUNSUPPORTED, "ndm exceeds max_ndm given to pwdf_create");
  return PWDF_OK;
}

int prof_id(pwdf_ctx *c, const std::string &name) {
  for (size_t i = 0; i < c->prof_names.size(); ++i)
    if (c->prof_names[i] == name) return (int)i;
  c->prof_names.push_back(name);
  c->prof_agg.emplace_back();
  return (int)c->prof_names.size() - 1;
}

hipEvent_t prof_event(pwdf_ctx *c) {
  if (c->prof_next == c->prof_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->prof_pool.push_back(e);
  }
  return c->prof_pool[c->prof_next++];
}

// Runs one launch; in profiling mode brackets it with events on the same stream.
template <class F>
pwdf_status step(pwdf_ctx *c, const char *name, double units, hipStream_t st, F &&launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (c->prof_on) {
    a = prof_event(c);
    b = prof_event(c);
    if (a) (void)hipEventRecord(a, st);
  }
  hipError_t e = launch();
  if (e != hipSuccess) return hip_fail(c, e, name);
  if (c->prof_on && a && b) {
    (void)hipEventRecord(b, st);
    c->prof_recs.push_back({prof_id(c, name), a, b, units});
  }
  return PWDF_OK;
}

// Fork/join of independent per-class launches over the internal streams (they
// write disjoint rows / blocks).  In profiling mode, and when the tune says so,
// everything stays on `st`.
struct Fork {
  pwdf_ctx *c;
  hipStream_t st;
  bool on;
  int next = 0;
  Fork(pwdf_ctx *c_, hipStream_t st_)
      : c(c_), st(st_), on(!c_->prof_on && c_->tune.fork && c_->aux[0] != nullptr) {
    if (!on) return;
    (void)hipEventRecord(c->ev_fork, st);
    for (int i = 0; i < kAux; ++i) (void)hipStreamWaitEvent(c->aux[i], c->ev_fork, 0);
  }
  hipStream_t stream() { return on ? c->aux[next++ % kAux] : st; }
  hipStream_t stream_at(int i) { return on ? c->aux[i % kAux] : st; }
  hipError_t join() {
    if (!on) return hipSuccess;
    hipError_t e = hipSuccess;
    for (int i = 0; i < kAux; ++i) {
      if ((e = hipEventRecord(c->ev_join[i], c->aux[i])) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(st, c->ev_join[i], 0)) != hipSuccess) return e;
    }
    return e;
  }
};

int np_L(const Plan &p, int L) { return p.L_p1[L] - p.L_p0[L]; }

// FP32-MFMA form: the per-class launches of one pass (pass 0: rho, 1: J) -- the
// tail (FP32 MFMA) of every class, then the head (FP64 MFMA) -- with the internal
// stream each goes to.  Default: that order, round robin over the streams.  With
// measured launch times (Tune::lpt): longest first, each onto the stream whose
// launches so far add up to the least time, so that no long launch starts last
// and runs alone at the end of the pass.
struct ClassLaunch {
  int head, L, stream;
};

std::vector<ClassLaunch> class_schedule(const Plan &p, const Dev &d, const Tune &t, int pass) {
  std::vector<ClassLaunch> v;
  std::vector<double> cost;
  for (int head = 0; head < 2; ++head)
    for (int L = 0; L <= 2 * kMaxL; ++L) {
      if (np_L(p, L) <= 0 || (head && d.npts_head <= 0)) continue;
      v.push_back({head, L, (int)v.size() % kAux});
      cost.push_back(t.cost[2 * pass + head][L]);
    }
  if (!t.lpt) return v;
  std::vector<int> idx(v.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  double load[kAux] = {};
  std::vector<ClassLaunch> out;
  for (int i : idx) {
    int s = 0;
    for (int k = 1; k < kAux; ++k)
      if (load[k] < load[s]) s = k;
    load[s] += cost[i];
    out.push_back({v[i].head, v[i].L, s});
  }
  return out;
}

// Algorithmic flops of one pair-G pass over the classes L in [L0, L1]: 8(L+1)+4
// per (unique pair, G of the half space, density) in the factored form.
double pass_flops(const Plan &p, int L0, int L1, int ndm) {
  double f = 0.0;
  for (int L = L0; L <= L1; ++L) f += p.pairG_L[L] * (8.0 * (L + 1) + 4.0);
  return f * ndm;
}

// Algorithmic flops of the density transform (or, the same count, of the back
// transform) over all pairs and ndm densities: per pair of class (la, lb), two
// per term of sum_{ab} D_ab E^x E^y E^z (one term per Hermite index t of each
// Cartesian element (a, b)), and two per entry of the Hermite -> relative-monomial
// blocks of every degree <= la + lb.
double pair_transform_flops(const Plan &p, int ndm) {
  double f = 0.0;
  for (int la = 0; la <= kMaxL; ++la)
    for (int lb = 0; lb <= la; ++lb) {
      const int cl = la * 4 + lb;
      if (p.cls_b1[cl] <= p.cls_b0[cl]) continue;
      double per = 0.0;
      for (int ax = la; ax >= 0; --ax)
        for (int ay = la - ax; ay >= 0; --ay)
          for (int bx = lb; bx >= 0; --bx)
            for (int by = lb - bx; by >= 0; --by) {
              const int az = la - ax - ay, bz = lb - bx - by;
              per += 2.0 * (ax + bx + 1) * (ay + by + 1) * (az + bz + 1);
            }
      for (int d = 0; d <= la + lb; ++d) per += 2.0 * ncart(d) * ncart(d);
      f += per * (double)(p.blocks[p.cls_b1[cl] - 1].p1 - p.blocks[p.cls_b0[cl]].p0);
    }
  return f * ndm;
}

double cls_pairs(const Plan &p, int cl) {
  return (double)(p.blocks[p.cls_b1[cl] - 1].p1 - p.blocks[p.cls_b0[cl]].p0);
}

// transform .. reduce (Dblk already holds D(L)); EJ device [ndm], or null to
// leave the energy partials for the J(k) launch
pwdf_status run_mid_rho(pwdf_ctx *c, int ndm, double *EJ, hipStream_t st) {
  const Plan &p = c->plan;
  const Dev &d = c->dev;
  const double nGh = (double)(p.nG_full / 2);
  pwdf_status s;
  char name[32];
  if ((s = step(c, "transform", pair_transform_flops(p, ndm), st, [&] { return launch_transform_all(d, ndm, st); })) !=
      PWDF_OK)
    return s;
  if (d.fp32) {
    Fork f(c, st);
    for (const ClassLaunch &cl : class_schedule(p, d, c->tune, 0)) {
      const int L = cl.L;
      hipStream_t ss = f.stream_at(cl.stream);
      std::snprintf(name, sizeof name, cl.head ? "rho_head_L%d" : "rho_mfma_L%d", L);
      if (cl.head)
        s = step(c, name, p.pairG_head_L[L] * ndm, ss, [&] { return launch_rho_head_L(d, L, ndm, ss); });
      else
        s = step(c, name, (p.pairG_L[L] - p.pairG_head_L[L]) * ndm, ss,
                 [&] { return launch_rho_mfma_L(d, L, ndm, ss); });
      if (s != PWDF_OK) return s;
    }
    if (hipError_t e = f.join()) return hip_fail(c, e, "join");
  } else {
    Fork f(c, st);
    for (int g = 0; g < 2; ++g) {
      if (!jpass_group_nonempty(d, g)) continue;
      hipStream_t ss = f.stream();
      if ((s = step(c, g ? "rho_hi" : "rho_lo", pass_flops(p, g ? 3 : 0, g ? 2 * kMaxL : 2, ndm), ss,
                    [&] { return launch_rho_group(d, g, ndm, ss); })) != PWDF_OK)
        return s;
    }
    if (hipError_t e = f.join()) return hip_fail(c, e, "join");
  }
  if (d.ndd == 0)
    return step(c, "reduce", (double)p.nslot() * ndm, st, [&] { return launch_reduce(d, ndm, EJ, st); });
  // compact/diffuse classification: the reduce gives rho_C; then rho_D of the DD
  // pairs, the combined potentials V_C and V_D and the energy partials
  if ((s = step(c, "reduce", (double)p.nslot() * ndm, st, [&] { return launch_reduce(d, ndm, nullptr, st); })) !=
      PWDF_OK)
    return s;
  if (d.gpw) {
    if ((s = step(c, "gpw_rho", (double)d.gpts * ndm, st, [&] { return launch_gpw_rho(d, ndm, st); })) != PWDF_OK)
      return s;
  } else if ((s = step(c, "rho_dd", (double)d.ndd * nGh * ndm, st, [&] { return launch_rho_dd(d, ndm, st); })) !=
             PWDF_OK) {
    return s;
  }
  if ((s = step(c, "combine_dd", (double)p.nslot() * ndm, st, [&] { return launch_combine_dd(d, ndm, st); })) !=
      PWDF_OK)
    return s;
  if (!EJ) return PWDF_OK;
  return step(c, "energy", (double)ndm, st, [&] { return launch_energy(d, ndm, EJ, st); });
}

pwdf_status run_to_rho(pwdf_ctx *c, int ndm, const double *Dk, double *EJ, hipStream_t st) {
  const Plan &p = c->plan;
  const Dev &d = c->dev;
  pwdf_status s;
  const double nsup = (double)(c->dk_layout == PWDF_DK_PACKED ? p.nDp_support : p.nD_support);
  if ((s = step(c, "phase_d", nsup * p.nk * ndm, st,
                [&] { return launch_phase_d(d, Dk, ndm, st); })) != PWDF_OK)
    return s;
  return run_mid_rho(c, ndm, EJ, st);
}

// J moments of both class groups (FP64) or per class (FP32-MFMA); force = true
// gives the degree L+1 moments of the gradient
pwdf_status run_moments(pwdf_ctx *c, int ndm, bool force, hipStream_t st) {
  const Plan &p = c->plan;
  const Dev &d = c->dev;
  const double nGh = (double)(p.nG_full / 2);
  pwdf_status s;
  char name[32];
  Fork f(c, st);
  if (d.fp32 && !force) {
    for (const ClassLaunch &cl : class_schedule(p, d, c->tune, 1)) {
      const int L = cl.L;
      hipStream_t ss = f.stream_at(cl.stream);
      std::snprintf(name, sizeof name, cl.head ? "jpass_head_L%d" : "jpass_mfma_L%d", L);
      if (cl.head)
        s = step(c, name, p.pairG_head_L[L] * ndm, ss, [&] { return launch_jpass_head_L(d, L, ndm, ss); });
      else
        s = step(c, name, (p.pairG_L[L] - p.pairG_head_L[L]) * ndm, ss,
                 [&] { return launch_jpass_mfma_L(d, L, ndm, ss); });
      if (s != PWDF_OK) return s;
    }
  } else {
    for (int g = 0; g < 2; ++g) {
      if (!jpass_group_nonempty(d, g)) continue;
      hipStream_t ss = f.stream();
      // force moments cost one degree more than the class's J moments
      const double fl = force ? pass_flops(p, g ? 3 : 0, g ? 2 * kMaxL : 2, ndm) +
                                    8.0 * nGh * ndm * (g ? np_L(p, 3) + np_L(p, 4) + np_L(p, 5) + np_L(p, 6)
                                                         : np_L(p, 0) + np_L(p, 1) + np_L(p, 2))
                              : pass_flops(p, g ? 3 : 0, g ? 2 * kMaxL : 2, ndm);
      const char *nm = force ? (g ? "jforce_hi" : "jforce_lo") : (g ? "jpass_hi" : "jpass_lo");
      if ((s = step(c, nm, fl, ss, [&] { return launch_jpass_group(d, g, force, ndm, ss); })) != PWDF_OK) return s;
    }
  }
  if (hipError_t e = f.join()) return hip_fail(c, e, "join");
  return PWDF_OK;
}

// (wprep) .. back transform: Jblk from V
pwdf_status run_mid_j(pwdf_ctx *c, int ndm, hipStream_t st) {
  const Plan &p = c->plan;
  const Dev &d = c->dev;
  pwdf_status s;
  if (d.fp32 && (s = step(c, "wprep", (double)p.nslot() * ndm, st, [&] { return launch_wprep(d, ndm, st); })) !=
                    PWDF_OK)
    return s;
  if ((s = run_moments(c, ndm, false, st)) != PWDF_OK) return s;
  if (d.gpw) {
    if ((s = step(c, "gpw_j", (double)d.gpts * ndm, st, [&] { return launch_gpw_j(d, ndm, st); })) != PWDF_OK)
      return s;
  } else if (d.ndd > 0 && (s = step(c, "jpass_dd", (double)d.ndd * (p.nG_full / 2) * ndm, st,
                                    [&] { return launch_jpass_dd(d, false, ndm, st); })) != PWDF_OK) {
    return s;
  }
  if ((s = step(c, "back", pair_transform_flops(p, ndm), st, [&] { return launch_back_all(d, ndm, st); })) !=
      PWDF_OK)
    return s;
  if (!d.gpw) return PWDF_OK;
  // GPW route: the DD pairs' J blocks, integrated on the grid, join J(L)
  return step(c, "gpw_add", (double)d.ndd * ndm, st, [&] { return launch_gpw_add(d, ndm, st); });
}

// EJ: device [ndm] summed by the J(k) launch from the energy partials of the
// preceding reduce (which was given EJ = null), or null
pwdf_status run_from_V(pwdf_ctx *c, int ndm, double *Jk, double *EJ, hipStream_t st) {
  const Plan &p = c->plan;
  const Dev &d = c->dev;
  pwdf_status s;
  if ((s = run_mid_j(c, ndm, st)) != PWDF_OK) return s;
  if ((s = step(c, "fold_j", (double)p.eJ.size() * ndm, st, [&] { return launch_fold_j(d, ndm, st); })) != PWDF_OK)
    return s;
  return step(c, "phase_j", (double)p.nk * (double)(p.lightJ.size() + p.heavyJ.size()) * ndm, st,
              [&] { return launch_phase_j(d, ndm, Jk, EJ, st); });
}

pwdf_status enqueue_build(pwdf_ctx *c, int ndm, const double *Dk, double *Jk, double *EJ, hipStream_t st) {
  pwdf_status s;
  if ((s = run_to_rho(c, ndm, Dk, nullptr, st)) != PWDF_OK) return s;
  return run_from_V(c, ndm, Jk, EJ, st);
}

}  // namespace

extern "C" {

// Argument checks shared by pwdf_create and pwdf_plan_stats; fills `in`.
static pwdf_status make_input(PlanInput &in, const double lattice[9], int natm, const double *xyz, int nshell,
                              const int *shell_atom, const int *shell_l, const int *shell_nprim,
                              const double *exps, const double *coefs, const int kmesh[3], double omega,
                              const pwdf_screen *screen) {
  if (!lattice || !xyz || !shell_atom || !shell_l || !shell_nprim || !exps || !coefs || !kmesh || !screen)
    return fail(nullptr, PWDF_EINVAL, "NULL input pointer");
  if (natm < 1 || nshell < 1) return fail(nullptr, PWDF_EINVAL, "natm and nshell must be >= 1");
  for (int s = 0; s < nshell; ++s)
    if (shell_l[s] < 0 || shell_l[s] > kMaxL) return fail(nullptr, PWDF_EUNSUPPORTED, "shell l outside 0..3");
  std::memcpy(in.lattice, lattice, sizeof(in.lattice));
  in.natm = natm;
  in.xyz.assign(xyz, xyz + 3 * natm);
  in.nshell = nshell;
  in.sh_atom.assign(shell_atom, shell_atom + nshell);
  in.sh_l.assign(shell_l, shell_l + nshell);
  in.sh_nprim.assign(shell_nprim, shell_nprim + nshell);
  int nprim = 0;
  for (int s = 0; s < nshell; ++s) {
    if (shell_nprim[s] < 1) return fail(nullptr, PWDF_EINVAL, "shell_nprim must be >= 1");
    nprim += shell_nprim[s];
  }
  in.exps.assign(exps, exps + nprim);
  in.coefs.assign(coefs, coefs + nprim);
  for (int i = 0; i < 3; ++i) in.kmesh[i] = kmesh[i];
  in.omega = omega;
  in.eps_pair = screen->eps_pair;
  in.eps_G = screen->eps_G;
  in.r_max = screen->r_max;
  in.pair_gcut = screen->pair_gcut != 0 ? 1 : 0;
  if (!std::isfinite(screen->alpha_cut)) return fail(nullptr, PWDF_EINVAL, "alpha_cut must be finite");
  in.alpha_cut = screen->alpha_cut > 0.0 ? screen->alpha_cut : 0.0;
  in.dd_gpw = screen->dd_gpw != 0 ? 1 : 0;
  return PWDF_OK;
}

static void fill_stats(const Plan &p, pwdf_stats *out) {
  std::memset(out, 0, sizeof(*out));
  for (int cl = 0; cl < 16; ++cl) {
    int b0 = p.cls_b0[cl], b1 = p.cls_b1[cl];
    if (b1 > b0) out->npairs_by_class[cl] = p.blocks[b1 - 1].p1 - p.blocks[b0].p0;
  }
  out->nG = p.nG_full;
  out->npairs = p.npairs();
  out->nbf = p.nbf;
  out->nk = p.nk;
  out->nimg = p.nimg();
  out->nblocks = (int64_t)p.blocks.size();
  out->nseg = p.nseg();
  // per build and density: both passes over the G each pair sees (its cut
  // sphere, or the whole half space)
  out->pairG_evals = 2.0 * p.pairG_cut + 2.0 * (double)p.dd_q.size() * (double)(p.nG_full / 2);
  out->npairs_dd = (int64_t)p.dd_q.size();
  for (int i = 0; i < 3; ++i) out->gpw_grid[i] = p.gN[i];
  out->seg_len = p.seg_len;
  out->fork = 1;
  out->jk_support = (int64_t)(p.lightJ.size() + p.heavyJ.size());
  out->dk_support = p.nD_support;
  out->jk_layout = PWDF_JK_FULL;
  out->nG_head = p.npts_head;
  out->pairG_head = 2.0 * p.pairG_head;
}

pwdf_status pwdf_plan_stats(const double lattice[9], int natm, const double *xyz, int nshell, const int *shell_atom,
                            const int *shell_l, const int *shell_nprim, const double *exps, const double *coefs,
                            const int kmesh[3], double omega, const pwdf_screen *screen, pwdf_stats *out) {
  if (!out) return fail(nullptr, PWDF_EINVAL, "out is NULL");
  PlanInput in;
  pwdf_status s = make_input(in, lattice, natm, xyz, nshell, shell_atom, shell_l, shell_nprim, exps, coefs, kmesh,
                             omega, screen);
  if (s != PWDF_OK) return s;
  Plan p;
  std::string why;
  try {
    why = build_plan(in, 8, p);
  } catch (const std::bad_alloc &) {
    return fail(nullptr, PWDF_ENOMEM, "host allocation failed while building the plan");
  }
  if (!why.empty()) return fail(nullptr, plan_status(why), why);
  fill_stats(p, out);
  return PWDF_OK;
}

void pwdf_destroy(pwdf_ctx *c);

pwdf_status pwdf_create(pwdf_ctx **out, const double lattice[9], int natm, const double *xyz, int nshell,
                        const int *shell_atom, const int *shell_l, const int *shell_nprim, const double *exps,
                        const double *coefs, const int kmesh[3], double omega, const pwdf_screen *screen,
                        pwdf_precision prec, int max_ndm, int device) {
  if (!out) return fail(nullptr, PWDF_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_ndm < 1) return fail(nullptr, PWDF_EINVAL, "max_ndm must be >= 1");
  if (prec != PWDF_FP64 && prec != PWDF_FP32_MFMA) return fail(nullptr, PWDF_EUNSUPPORTED, "unknown precision");
  if (prec == PWDF_FP32_MFMA && max_ndm > 16)
    return fail(nullptr, PWDF_EUNSUPPORTED, "the FP32-MFMA form takes at most 16 densities per call");
  pwdf_ctx *c = new (std::nothrow) pwdf_ctx();
  if (!c) return fail(nullptr, PWDF_ENOMEM, "host allocation failed");
  {
    pwdf_status s = make_input(c->in, lattice, natm, xyz, nshell, shell_atom, shell_l, shell_nprim, exps, coefs,
                               kmesh, omega, screen);
    if (s != PWDF_OK) {
      delete c;
      return s;
    }
  }
  std::string why;
  try {
    why = build_plan(c->in, 8, c->plan);
  } catch (const std::bad_alloc &) {
    delete c;
    return fail(nullptr, PWDF_ENOMEM, "host allocation failed while building the plan");
  }
  if (!why.empty()) {
    delete c;
    return fail(nullptr, plan_status(why), why);
  }
  // the phase kernels stage the (n1+n2+n3) lcm(n1,n2,n3) phases in LDS
  if (c->plan.ptab.size() / 2 > 1024) {
    delete c;
    return fail(nullptr, PWDF_EUNSUPPORTED, "k-mesh too large: need (n1+n2+n3)*lcm(n1,n2,n3) <= 1024");
  }
  c->device = device;
  c->max_ndm = max_ndm;
  c->prec = prec;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) {
    delete c;
    return fail(nullptr, PWDF_EDEVICE, std::string("no HIP device: ") + hipGetErrorString(e));
  }
  if (device < 0 || device >= ndev) {
    delete c;
    return fail(nullptr, PWDF_EINVAL, "device ordinal out of range");
  }
  if ((e = hipSetDevice(device)) != hipSuccess) {
    delete c;
    return fail(nullptr, PWDF_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
  }
  // internal streams (default priority) and fork/join events
  bool ok = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; ok && i < kAux; ++i)
    ok = hipStreamCreateWithFlags(&c->aux[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&c->ev_join[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    pwdf_destroy(c);
    return fail(nullptr, PWDF_EDEVICE, "creating internal streams");
  }
  pwdf_status s = setup_device(c, Tune());
  if (s != PWDF_OK) {
    std::string m = c->err;
    pwdf_destroy(c);
    return fail(nullptr, s, m);
  }
  *out = c;
  return PWDF_OK;
}

pwdf_status pwdf_query(const pwdf_ctx *c, pwdf_stats *out) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_query: ctx is NULL");
  if (!out) return fail(const_cast<pwdf_ctx *>(c), PWDF_EINVAL, "pwdf_query: out is NULL");
  fill_stats(c->plan, out);
  out->seg_len = c->plan.seg_len;
  out->fork = c->tune.fork;
  out->jk_layout = c->jk_layout;
  if (c->dk_layout == PWDF_DK_PACKED) out->dk_support = c->plan.nDp_support;
  return PWDF_OK;
}

pwdf_status pwdf_set_jk_layout(pwdf_ctx *c, int layout) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_set_jk_layout: ctx is NULL");
  if (layout != PWDF_JK_FULL && layout != PWDF_JK_SUPPORT && layout != PWDF_JK_PACKED)
    return fail(c, PWDF_EINVAL, "layout must be PWDF_JK_FULL, PWDF_JK_SUPPORT or PWDF_JK_PACKED");
  if (layout != c->jk_layout) drop_graph(c);  // the captured J(k) launch has the old shape
  c->jk_layout = layout;
  c->dev.jk_layout = layout;
  return PWDF_OK;
}

pwdf_status pwdf_set_dk_layout(pwdf_ctx *c, int layout) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_set_dk_layout: ctx is NULL");
  if (layout != PWDF_DK_FULL && layout != PWDF_DK_PACKED)
    return fail(c, PWDF_EINVAL, "layout must be PWDF_DK_FULL or PWDF_DK_PACKED");
  if (layout != c->dk_layout) drop_graph(c);  // the captured D(k) launch reads the old layout
  c->dk_layout = layout;
  c->dev.dk_layout = layout;
  return PWDF_OK;
}

pwdf_status pwdf_set_fp32_head(pwdf_ctx *c, double weight) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_set_fp32_head: ctx is NULL");
  if (!(weight > 0.0 && weight <= 1.0)) return fail(c, PWDF_EINVAL, "head weight must be in (0, 1]");
  if (!c->ready) return not_ready(c);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  // the workspaces are rebuilt below: nothing may still be running on them
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
  set_head_weight(c->plan, weight);
  return setup_device(c, c->tune);
}

pwdf_status pwdf_get_jk_support(const pwdf_ctx *c, int *mu, int *nu) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_get_jk_support: ctx is NULL");
  const Plan &p = c->plan;
  size_t i = 0;
  for (const std::vector<int> *v : {&p.lightJ, &p.heavyJ})
    for (int e : *v) {
      if (mu) mu[i] = e / p.nbf;
      if (nu) nu[i] = e % p.nbf;
      ++i;
    }
  return PWDF_OK;
}

pwdf_status pwdf_check_input(pwdf_ctx *c, void *stream) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_check_input: ctx is NULL");
  if (!c->ready) return not_ready(c);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  int flag = 0;
  if ((e = hipMemcpyAsync(&flag, c->dev.nonfinite, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hip_fail(c, e, "reading the input flag");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(c, e, "sync");
  if (!flag) return PWDF_OK;
  if ((e = hipMemsetAsync(c->dev.nonfinite, 0, sizeof(int), st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return hip_fail(c, e, "clearing the input flag");
  return fail(c, PWDF_ENONFINITE, "a D(k) value on the pair support was not finite (NaN or inf) in a call since "
                                  "the last check; its results are not usable");
}

pwdf_status pwdf_build_j(pwdf_ctx *c, int ndm, const double *Dk, double *Jk, double *EJ, void *stream) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_build_j: ctx is NULL");
  pwdf_status s = validate_ndm(c, ndm);
  if (s != PWDF_OK) return s;
  if (!Dk || !Jk || !EJ) return fail(c, PWDF_EINVAL, "NULL buffer");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  c->blocks_ndm = 0;
  if ((s = enqueue_build(c, ndm, Dk, Jk, EJ, (hipStream_t)stream)) != PWDF_OK) return s;
  c->blocks_ndm = ndm;
  return PWDF_OK;
}

pwdf_status pwdf_build_j_graph(pwdf_ctx *c, int ndm, const double *Dk, double *Jk, double *EJ, void *stream) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_build_j_graph: ctx is NULL");
  pwdf_status s = validate_ndm(c, ndm);
  if (s != PWDF_OK) return s;
  if (!Dk || !Jk || !EJ) return fail(c, PWDF_EINVAL, "NULL buffer");
  if (c->prof_on) return fail(c, PWDF_ESTATE, "graph replay is not available in profiling mode");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  GraphCache &g = c->gc;
  if (!(g.exec && g.ndm == ndm && g.Dk == Dk && g.Jk == Jk && g.EJ == EJ)) {
    drop_graph(c);
    if ((e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(c, e, "begin capture");
    s = enqueue_build(c, ndm, Dk, Jk, EJ, c->cap);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->cap, &graph);
    if (s != PWDF_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e2 != hipSuccess) return hip_fail(c, e2, "end capture");
    hipGraphExec_t exec = nullptr;
    if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(c, e, "graph instantiate");
    }
    g.graph = graph;
    g.exec = exec;
    g.ndm = ndm;
    g.Dk = Dk;
    g.Jk = Jk;
    g.EJ = EJ;
  }
  c->blocks_ndm = 0;
  if ((e = hipGraphLaunch(g.exec, st)) != hipSuccess) return hip_fail(c, e, "graph launch");
  c->blocks_ndm = ndm;
  return PWDF_OK;
}

// Byte layout of the per-call workspaces of a J build for ndm densities inside
// one buffer (each piece 256-byte aligned); fills the pointers of d when base is
// not null and returns the bytes needed.
static size_t carve_build_ws(Dev &d, const Plan &p, int ndm, unsigned char *base) {
  size_t off = 0;
  auto take = [&](auto *&field, size_t count) {
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(field)>>;
    off = (off + 255) / 256 * 256;
    if (base) field = reinterpret_cast<T *>(base + off);
    off += std::max<size_t>(1, count) * sizeof(T);
  };
  const size_t M = (size_t)ndm;
  take(d.Dblk, M * p.nelem);
  take(d.Jblk, M * p.nelem);
  take(d.dhat, d.fp32 ? (size_t)std::max<int64_t>(1, d.d32_size) : M * d.dhat_size);
  take(d.yhat, M * d.yhat_size);
  take(d.part, M * d.nrows * part_cols(d));
  take(d.part2, M * d.ngroups * d.nslot);
  take(d.rho, M * d.nslot);
  take(d.Vc, M * d.nslot);
  take(d.Epart, M * d.nred_blocks);
  if (d.ndd > 0) {
    take(d.rhoD, M * d.nslot);
    take(d.rhoDp, M * d.dd_chunks * d.nslot);
    take(d.VDc, M * d.nslot);
    take(d.ydd, M * d.ndd * kDDStride);
  }
  if (d.gpw) {
    take(d.grid_r, M * d.gpts);
    take(d.grid_p, M * d.ngitems * 512);
    take(d.grid_a, M * gpw_a_size(d));
    take(d.grid_b, M * gpw_b_size(d));
    take(d.grid_c, M * gpw_c_size(d));
    take(d.gpw_part, M * d.ndd * kGpwEl);
  }
  take(d.Jfold, M * (size_t)std::max(1, d.nsegJ));
  if (d.npts_head > 0) take(d.parth, M * d.nrows_h * d.npts_head);
  if (d.fp32) {
    take(d.dh32, (size_t)std::max<int64_t>(1, d.d32_size));
    take(d.wre, (size_t)d.nslot * d.ncolsW);
    take(d.wim, (size_t)d.nslot * d.ncolsW);
    if (d.npts_head > 0) {
      take(d.wre64, (size_t)d.npts_head * d.ncolsW);
      take(d.wim64, (size_t)d.npts_head * d.ncolsW);
    }
  }
  return off;
}

pwdf_status pwdf_build_j_noalloc(pwdf_ctx *c, int ndm, const double *Dk, double *Jk, double *EJ, void *stream) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_build_j_noalloc: ctx is NULL");
  pwdf_status s = validate_ndm(c, ndm);
  if (s != PWDF_OK) return s;
  if (!Dk || !Jk || !EJ) return fail(c, PWDF_EINVAL, "NULL buffer");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  Dev d = c->dev;
  const size_t need = carve_build_ws(d, c->plan, ndm, nullptr);
  if (need > kStaticScratchBytes) {
    char m[256];
    std::snprintf(m, sizeof m,
                  "pwdf_build_j_noalloc: %d densities of this plan need %zu bytes of workspace, the static "
                  "scratch holds %zu (use pwdf_build_j, or fewer densities per call)",
                  ndm, need, (size_t)kStaticScratchBytes);
    return fail(c, PWDF_EUNSUPPORTED, m);
  }
  void *base = nullptr;
  if ((e = static_scratch(c->device, &base)) != hipSuccess) return hip_fail(c, e, "static scratch address");
  carve_build_ws(d, c->plan, ndm, static_cast<unsigned char *>(base));
  hipStream_t st = (hipStream_t)stream;
  // the FP32-MFMA operand columns past the densities must read as zeros: the
  // scratch holds whatever the previous call on this device left there
  if (d.fp32 && (e = launch_zero_f32(d.dh32, std::max<int64_t>(1, d.d32_size), st)) != hipSuccess)
    return hip_fail(c, e, "clearing the operand buffer");
  // the launch sequence of pwdf_build_j on the scratch-backed workspaces
  const Dev saved = c->dev;
  c->dev = d;
  s = enqueue_build(c, ndm, Dk, Jk, EJ, st);
  c->dev = saved;
  c->blocks_ndm = 0;  // the blocks went to the shared scratch
  return s;
}

pwdf_status pwdf_energy_real(pwdf_ctx *c, int ndm, double *ER, void *stream) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_energy_real: ctx is NULL");
  if (!ER) return fail(c, PWDF_EINVAL, "NULL buffer");
  if (ndm < 1 || ndm > c->blocks_ndm) {
    char m[256];
    std::snprintf(m, sizeof m,
                  "pwdf_energy_real: the workspace holds the D(L) and J(L) blocks of %d densities (those of the "
                  "last pwdf_build_j or pwdf_build_j_graph call; any other call replaces them), %d asked",
                  c->blocks_ndm, ndm);
    return fail(c, PWDF_ESTATE, m);
  }
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  if ((e = launch_energy_real(c->dev, ndm, c->ERpart, ER, (hipStream_t)stream)) != hipSuccess)
    return hip_fail(c, e, "real-space energy");
  return PWDF_OK;
}

pwdf_status pwdf_get_rhoG(pwdf_ctx *c, int ndm, const double *Dk, double *rhoG, int *miller, void *stream) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_get_rhoG: ctx is NULL");
  pwdf_status s = validate_ndm(c, ndm);
  if (s != PWDF_OK) return s;
  if (!Dk || !rhoG) return fail(c, PWDF_EINVAL, "NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  c->blocks_ndm = 0;
  if ((s = run_to_rho(c, ndm, Dk, c->Escr, st)) != PWDF_OK) return s;
  // the valid slots gathered on the device, on the caller's stream
  if ((e = launch_gather_rho(c->dev, ndm, reinterpret_cast<double2 *>(rhoG), st)) != hipSuccess)
    return hip_fail(c, e, "gathering rho");
  const Plan &p = c->plan;
  if (miller)
    for (size_t i = 0; i < p.valid_slots.size(); ++i)
      for (int x = 0; x < 3; ++x) miller[3 * i + x] = p.slot_miller[3 * (size_t)p.valid_slots[i] + x];
  return PWDF_OK;
}

pwdf_status pwdf_grad(pwdf_ctx *c, int ndm, const double *Dk, double *dEdR, double *EJ, void *stream) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_grad: ctx is NULL");
  pwdf_status s = validate_ndm(c, ndm);
  if (s != PWDF_OK) return s;
  if (!Dk || !dEdR) return fail(c, PWDF_EINVAL, "NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  // energy path (rho, V) in the context's precision; the adjoint moments and the
  // centre-derivative contraction run in FP64
  c->blocks_ndm = 0;
  if ((s = run_to_rho(c, ndm, Dk, EJ ? EJ : c->Escr, st)) != PWDF_OK) return s;
  const Plan &p = c->plan;
  const Dev &d = c->dev;
  char name[32];
  if ((s = run_moments(c, ndm, true, st)) != PWDF_OK) return s;
  if (d.ndd > 0 && (s = step(c, "jforce_dd", (double)d.ndd * (p.nG_full / 2) * ndm, st,
                             [&] { return launch_jpass_dd(d, true, ndm, st); })) != PWDF_OK)
    return s;
  {
    Fork f(c, st);
    for (int la = 0; la <= kMaxL; ++la)
      for (int lb = 0; lb <= la; ++lb) {
        int cl = la * 4 + lb;
        if (p.cls_b1[cl] <= p.cls_b0[cl]) continue;
        std::snprintf(name, sizeof name, "fback_%d%d", la, lb);
        hipStream_t ss = f.stream();
        if ((s = step(c, name, cls_pairs(p, cl) * ndm, ss,
                      [&] { return launch_force_back_cls(d, la, lb, ndm, ss); })) != PWDF_OK)
          return s;
      }
    if ((e = f.join()) != hipSuccess) return hip_fail(c, e, "join");
  }
  return step(c, "force_atoms", (double)d.natm * 3 * ndm, st, [&] { return launch_force_atoms(d, ndm, dEdR, st); });
}

// ---------------------------------------------------------------------------
// autotuning
// ---------------------------------------------------------------------------

static std::string tune_key(const pwdf_ctx *c, int ndm) {
  char k[256];
  std::snprintf(k, sizeof k, "gfx950|%s|nG=%lld|pairs=%d|nbf=%d|nk=%d|ndm=%d", c->prec == PWDF_FP64 ? "fp64" : "fp32",
                (long long)c->plan.nG_full, c->plan.npairs(), c->plan.nbf, c->plan.nk, ndm);
  return k;
}

// Segment lengths the kernels are built for, per precision form.
static std::vector<int> seg_lengths(int prec) {
  // the FP32-MFMA pair-G kernels walk the compact point list: the segment length
  // only sets the slot layout of rho and V there
  return prec == PWDF_FP32_MFMA ? std::vector<int>{8} : std::vector<int>{4, 5, 8, 16};
}

static bool load_tune(const char *path, const std::string &key, Tune &t) {
  if (!path) return false;
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char line[2048];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    char kbuf[512];
    int seg;
    int n = 0;
    if (std::sscanf(line, "%511s %d%n", kbuf, &seg, &n) < 2 || key != kbuf) continue;
    Tune u;
    u.seg_len = seg;
    const char *q = line + n;
    bool good = true;
    for (int L = 0; L <= kMaxLsum && good; ++L) {
      int m = 0;
      good = std::sscanf(q, "%lf%n", &u.mrho[L], &m) == 1;
      q += m;
    }
    for (int L = 0; L <= kMaxLsum && good; ++L) {
      int m = 0;
      good = std::sscanf(q, "%lf%n", &u.mj[L], &m) == 1;
      q += m;
    }
    if (good) {
      int f = 1, m = 0;
      if (std::sscanf(q, "%d%n", &f, &m) == 1) {
        u.fork = f != 0;
        q += m;
        // optional: the launch order flag and the measured per-class launch times
        Tune w = u;
        int lpt = 0;
        bool more = std::sscanf(q, "%d%n", &lpt, &m) == 1;
        if (more) q += m;
        for (int i = 0; i < 4 && more; ++i)
          for (int L = 0; L <= kMaxLsum && more; ++L) {
            more = std::sscanf(q, "%lf%n", &w.cost[i][L], &m) == 1;
            q += m;
          }
        if (more) {
          w.lpt = lpt != 0;
          u = w;
        }
      }
      t = u;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

static void save_tune(const char *path, const std::string &key, const Tune &t) {
  if (!path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d", key.c_str(), t.seg_len);
  for (int L = 0; L <= kMaxLsum; ++L) std::fprintf(f, " %.6g", t.mrho[L]);
  for (int L = 0; L <= kMaxLsum; ++L) std::fprintf(f, " %.6g", t.mj[L]);
  std::fprintf(f, " %d %d", t.fork, t.lpt);
  for (int i = 0; i < 4; ++i)
    for (int L = 0; L <= kMaxLsum; ++L) std::fprintf(f, " %.6g", t.cost[i][L]);
  std::fprintf(f, "\n");
  std::fclose(f);
}

// Per-kernel milliseconds of the tunable part (transform .. back transform), one
// warm-up and `reps` profiled repetitions on the tuning stream.
static pwdf_status time_tunable(pwdf_ctx *c, int ndm, int reps, std::vector<std::pair<std::string, double>> &out,
                                double &total) {
  pwdf_status s;
  hipError_t e;
  if ((e = hipMemsetAsync(c->dev.Dblk, 0, sizeof(double) * (size_t)ndm * c->plan.nelem, c->cap)) != hipSuccess)
    return hip_fail(c, e, "tune clear");
  if ((s = run_mid_rho(c, ndm, c->Escr, c->cap)) != PWDF_OK) return s;
  if ((s = run_mid_j(c, ndm, c->cap)) != PWDF_OK) return s;
  if ((e = hipStreamSynchronize(c->cap)) != hipSuccess) return hip_fail(c, e, "tune sync");
  c->prof_on = true;
  c->prof_recs.clear();
  c->prof_next = 0;
  for (auto &a : c->prof_agg) a = ProfAgg();
  for (int r = 0; r < reps; ++r) {
    if ((s = run_mid_rho(c, ndm, c->Escr, c->cap)) != PWDF_OK) break;
    if ((s = run_mid_j(c, ndm, c->cap)) != PWDF_OK) break;
  }
  c->prof_on = false;
  if (s != PWDF_OK) return s;
  total = 0.0;
  out.clear();
  for (const ProfRec &r : c->prof_recs) {
    if ((e = hipEventSynchronize(r.b)) != hipSuccess) return hip_fail(c, e, "tune events");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    total += ms / reps;
    bool hit = false;
    for (auto &kv : out)
      if (kv.first == c->prof_names[r.id]) {
        kv.second += ms / reps;
        hit = true;
      }
    if (!hit) out.push_back({c->prof_names[r.id], ms / reps});
  }
  c->prof_recs.clear();
  c->prof_next = 0;
  return PWDF_OK;
}

// Wall time per repetition of the tunable part (transform .. back transform)
// with eager launches on the tuning stream (the FP32-MFMA form's tuner).
static pwdf_status time_total_eager(pwdf_ctx *c, int ndm, int reps, double &ms_out) {
  pwdf_status s;
  hipError_t e;
  if ((e = hipMemsetAsync(c->dev.Dblk, 0, sizeof(double) * (size_t)ndm * c->plan.nelem, c->cap)) != hipSuccess)
    return hip_fail(c, e, "tune clear");
  hipEvent_t a = prof_event(c), b = prof_event(c);
  if (!a || !b) return fail(c, PWDF_EDEVICE, "tune events");
  for (int r = -1; r < reps; ++r) {  // r = -1: warm-up
    if (r == 0 && (e = hipEventRecord(a, c->cap)) != hipSuccess) return hip_fail(c, e, "tune events");
    if ((s = run_mid_rho(c, ndm, c->Escr, c->cap)) != PWDF_OK) return s;
    if ((s = run_mid_j(c, ndm, c->cap)) != PWDF_OK) return s;
  }
  if ((e = hipEventRecord(b, c->cap)) != hipSuccess || (e = hipEventSynchronize(b)) != hipSuccess)
    return hip_fail(c, e, "tune events");
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  c->prof_next = 0;
  ms_out = ms / reps;
  return PWDF_OK;
}

// Wall time per repetition of the tunable part (transform .. back transform) as
// a graph replayed on the tuning stream, the launches of one pass overlapping
// as the tune's fork setting makes them in a build.  The FP32-MFMA form times
// eager launches instead (time_total_eager).
static pwdf_status time_total(pwdf_ctx *c, int ndm, int reps, double &ms_out) {
  if (c->prec == PWDF_FP32_MFMA) return time_total_eager(c, ndm, reps, ms_out);
  pwdf_status s;
  hipError_t e;
  if ((e = hipMemsetAsync(c->dev.Dblk, 0, sizeof(double) * (size_t)ndm * c->plan.nelem, c->cap)) != hipSuccess)
    return hip_fail(c, e, "tune clear");
  if ((e = hipStreamSynchronize(c->cap)) != hipSuccess) return hip_fail(c, e, "tune sync");
  if ((e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return hip_fail(c, e, "tune capture");
  s = run_mid_rho(c, ndm, c->Escr, c->cap);
  if (s == PWDF_OK) s = run_mid_j(c, ndm, c->cap);
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->cap, &graph);
  if (s != PWDF_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e2 != hipSuccess) return hip_fail(c, e2, "tune capture");
  hipGraphExec_t exec = nullptr;
  if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(c, e, "tune graph");
  }
  hipEvent_t a = prof_event(c), b = prof_event(c);
  if (!a || !b) e = hipErrorOutOfMemory;
  for (int r = -1; r < reps && e == hipSuccess; ++r) {  // r = -1: warm-up
    if (r == 0) e = hipEventRecord(a, c->cap);
    if (e == hipSuccess) e = hipGraphLaunch(exec, c->cap);
  }
  if (e == hipSuccess) e = hipEventRecord(b, c->cap);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0.f;
  if (e == hipSuccess) (void)hipEventElapsedTime(&ms, a, b);
  (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  c->prof_next = 0;
  if (e != hipSuccess) return hip_fail(c, e, "tune timing");
  ms_out = ms / reps;
  return PWDF_OK;
}

static double kernel_ms(const std::vector<std::pair<std::string, double>> &v, const std::string &name) {
  for (auto &kv : v)
    if (kv.first == name) return kv.second;
  return 0.0;
}

pwdf_status pwdf_autotune(pwdf_ctx *c, int ndm, const char *cache_path) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_autotune: ctx is NULL");
  pwdf_status s = validate_ndm(c, ndm);
  if (s != PWDF_OK) return s;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  // the workspaces are rebuilt below: nothing may still be running on them
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
  c->blocks_ndm = 0;
  const std::string key = tune_key(c, ndm);
  Tune best;
  if (load_tune(cache_path, key, best)) {
    const std::vector<int> ok = seg_lengths(c->prec);
    if (std::find(ok.begin(), ok.end(), best.seg_len) == ok.end())
      return fail(c, PWDF_EINVAL, "tune cache: segment length not supported");
    if (best.seg_len != c->plan.seg_len) build_segments(c->plan, best.seg_len);
    return setup_device(c, best);
  }
  const bool was_prof = c->prof_on;
  c->prof_on = false;
  // Each candidate: the workspaces set up for it, two timings of graph replays,
  // the shorter kept.
  auto measure = [&](const Tune &t, double &ms) -> pwdf_status {
    if (t.seg_len != c->plan.seg_len) build_segments(c->plan, t.seg_len);
    pwdf_status r = setup_device(c, t);
    double a = 0.0, b = 0.0;
    if (r == PWDF_OK) r = time_total(c, ndm, 5, a);
    if (r == PWDF_OK) r = time_total(c, ndm, 5, b);
    ms = std::min(a, b);
    return r;
  };
  // 1. segment length and a common multiplier (1/2, 1, 2) of the chunk counts of
  // the pair-G passes: for FP64 searched jointly (the best multiplier depends on
  // the segment length), for the FP32-MFMA form the segment length at 1 and then
  // the multipliers for it; a warm-up, every candidate timed once, then the
  // three best timed again in reverse order, each keeping its shortest time
  const std::vector<int> segs = seg_lengths(c->prec);
  struct Cand {
    Tune t;
    double ms;
  };
  std::vector<Cand> cands;
  auto add = [&](int sl, double m) {
    Cand k;
    k.t.seg_len = sl;
    for (int L = 0; L <= kMaxLsum; ++L) k.t.mrho[L] = k.t.mj[L] = m;
    k.ms = 1e300;
    cands.push_back(k);
  };
  auto by_time = [](const Cand &x, const Cand &y) { return x.ms < y.ms; };
  const bool joint = c->prec == PWDF_FP64;
  for (int sl : segs)
    for (double m : {1.0, 0.5, 2.0})
      if (joint || m == 1.0) add(sl, m);
  {
    double ms = 0.0;
    if ((s = measure(cands.back().t, ms)) != PWDF_OK) return s;
  }
  for (Cand &k : cands)
    if ((s = measure(k.t, k.ms)) != PWDF_OK) return s;
  std::stable_sort(cands.begin(), cands.end(), by_time);
  if (!joint) {
    // FP32-MFMA form: the multipliers for the fastest segment length only
    const int sl = cands[0].t.seg_len;
    const size_t n0 = cands.size();
    add(sl, 0.5);
    add(sl, 2.0);
    for (size_t i = n0; i < cands.size(); ++i)
      if ((s = measure(cands[i].t, cands[i].ms)) != PWDF_OK) return s;
    std::stable_sort(cands.begin(), cands.end(), by_time);
  }
  for (int i = std::min<int>(3, (int)cands.size()) - 1; i >= 0; --i) {
    double ms = 0.0;
    if ((s = measure(cands[i].t, ms)) != PWDF_OK) return s;
    cands[i].ms = std::min(cands[i].ms, ms);
  }
  std::stable_sort(cands.begin(), cands.end(), by_time);
  best = cands[0].t;
  double best_t = cands[0].ms;
  if (best.seg_len != c->plan.seg_len) build_segments(c->plan, best.seg_len);
  Tune cand = best;
  // 2. FP32-MFMA form (one launch per class): each class keeps the multiplier
  // with its shortest kernel, timed one launch at a time, and the result is kept
  // only if it also wins when the classes overlap
  if (c->prec == PWDF_FP32_MFMA) {
    const double mults[] = {0.25, 0.5, 1.0, 2.0, 4.0};
    double brho[kMaxLsum + 1], bj[kMaxLsum + 1];
    for (int L = 0; L <= kMaxLsum; ++L) brho[L] = bj[L] = 1e300;
    std::vector<std::pair<std::string, double>> per;
    for (double m : mults) {
      Tune t = best;
      for (int L = 0; L <= kMaxLsum; ++L) {
        t.mrho[L] *= m;
        t.mj[L] *= m;
      }
      if ((s = setup_device(c, t)) != PWDF_OK) return s;
      double tot = 0.0;
      if ((s = time_tunable(c, ndm, 3, per, tot)) != PWDF_OK) return s;
      char name[32];
      for (int L = 0; L <= 2 * kMaxL; ++L) {
        if (np_L(c->plan, L) <= 0) continue;
        std::snprintf(name, sizeof name, "rho_mfma_L%d", L);
        const double tr = kernel_ms(per, name);
        std::snprintf(name, sizeof name, "jpass_mfma_L%d", L);
        const double tj = kernel_ms(per, name);
        if (tr < brho[L]) {
          brho[L] = tr;
          cand.mrho[L] = t.mrho[L];
        }
        if (tj < bj[L]) {
          bj[L] = tj;
          cand.mj[L] = t.mj[L];
        }
      }
    }
    if ((s = setup_device(c, cand)) != PWDF_OK) return s;
    double t_cand = 0.0;
    if ((s = time_total(c, ndm, 5, t_cand)) != PWDF_OK) return s;
    if (t_cand > best_t) cand = best;
  }
  // 2b. FP64: the J pass's multiplier apart from rho's (the passes split the work
  // along different axes: rho chunks the pairs, J the G segments), then rho's
  // around the joint choice, then both passes' multipliers of the classes L >= 3
  // (their own launches, wave-per-pair bodies of a larger register footprint)
  // apart from those of L <= 2; a variation is kept only when it is at least 1 %
  // faster than the current choice (two timings each, the shorter kept)
  if (c->prec == PWDF_FP64) {
    const double vars[][2] = {{1.0, 0.5}, {1.0, 2.0}, {0.75, 1.0}, {1.5, 1.0}};
    for (const auto &v : vars) {
      Tune t = cand;
      for (int L = 0; L <= kMaxLsum; ++L) {
        t.mrho[L] *= v[0];
        t.mj[L] *= v[1];
      }
      double ms = 0.0;
      if ((s = measure(t, ms)) != PWDF_OK) return s;
      if (ms < 0.99 * best_t) {
        cand = t;
        best_t = ms;
      }
    }
    bool high = false;
    for (int L = 3; L <= kMaxLsum; ++L) high = high || np_L(c->plan, L) > 0;
    for (double m : {0.5, 2.0}) {
      if (!high) break;
      Tune t = cand;
      for (int L = 3; L <= kMaxLsum; ++L) {
        t.mrho[L] *= m;
        t.mj[L] *= m;
      }
      double ms = 0.0;
      if ((s = measure(t, ms)) != PWDF_OK) return s;
      if (ms < 0.99 * best_t) {
        cand = t;
        best_t = ms;
      }
    }
  }
  // 3. the independent launches of a pass overlapping on the internal streams,
  // or following each other on one stream: timed back to back.  The FP32-MFMA
  // form first measures its per-class launch times (one launch at a time) and
  // also times the overlapping launches ordered by them (class_schedule)
  if ((s = setup_device(c, cand)) != PWDF_OK) return s;
  if (c->prec == PWDF_FP32_MFMA) {
    std::vector<std::pair<std::string, double>> per;
    double tot = 0.0;
    if ((s = time_tunable(c, ndm, 3, per, tot)) != PWDF_OK) return s;
    char name[32];
    const char *fmt[4] = {"rho_mfma_L%d", "rho_head_L%d", "jpass_mfma_L%d", "jpass_head_L%d"};
    for (int i = 0; i < 4; ++i)
      for (int L = 0; L <= kMaxLsum; ++L) {
        std::snprintf(name, sizeof name, fmt[i], L);
        cand.cost[i][L] = kernel_ms(per, name);
      }
    c->tune = cand;
  }
  {
    // variants (fork, lpt): overlapping in class order, overlapping longest
    // first (FP32-MFMA form), in order; each timed twice, in both orders
    std::vector<std::pair<int, int>> vars = {{1, 0}, {0, 0}};
    if (c->prec == PWDF_FP32_MFMA) vars.push_back({1, 1});
    std::vector<double> best_v(vars.size(), 1e300);
    for (int rep = 0; rep < 2; ++rep)
      for (size_t k = 0; k < vars.size(); ++k) {
        const size_t i = rep ? vars.size() - 1 - k : k;
        c->tune.fork = vars[i].first;
        c->tune.lpt = vars[i].second;
        double ms = 0.0;
        if ((s = time_total(c, ndm, 5, ms)) != PWDF_OK) return s;
        best_v[i] = std::min(best_v[i], ms);
      }
    size_t b = 0;
    for (size_t i = 1; i < vars.size(); ++i)
      if (best_v[i] < best_v[b]) b = i;
    cand.fork = vars[b].first;
    cand.lpt = vars[b].second;
    c->tune.fork = cand.fork;
    c->tune.lpt = cand.lpt;
  }
  c->prof_on = was_prof;
  save_tune(cache_path, key, cand);
  return PWDF_OK;
}

pwdf_status pwdf_profile_enable(pwdf_ctx *c, int on) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_profile_enable: ctx is NULL");
  c->prof_on = on != 0;
  c->prof_recs.clear();
  c->prof_next = 0;
  for (auto &a : c->prof_agg) a = ProfAgg();
  return PWDF_OK;
}

pwdf_status pwdf_profile_read(pwdf_ctx *c, pwdf_kprof *out, int max, int *n) {
  if (!c) return fail(nullptr, PWDF_EINVAL, "pwdf_profile_read: ctx is NULL");
  if (!n) return fail(c, PWDF_EINVAL, "pwdf_profile_read: n is NULL");
  (void)hipSetDevice(c->device);
  for (const ProfRec &r : c->prof_recs) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return hip_fail(c, e, "profile read");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return hip_fail(c, e, "profile read");
    ProfAgg &g = c->prof_agg[r.id];
    g.launches += 1;
    g.ms += ms;
    g.units += r.units;
  }
  c->prof_recs.clear();
  c->prof_next = 0;
  int k = 0;
  for (size_t i = 0; i < c->prof_names.size(); ++i) {
    if (c->prof_agg[i].launches == 0) continue;
    if (out && k < max) {
      std::memset(&out[k], 0, sizeof(out[k]));
      std::snprintf(out[k].name, sizeof(out[k].name), "%s", c->prof_names[i].c_str());
      out[k].launches = c->prof_agg[i].launches;
      out[k].ms = c->prof_agg[i].ms;
      out[k].units = c->prof_agg[i].units;
    }
    ++k;
  }
  *n = k;
  return PWDF_OK;
}

const char *pwdf_last_error(const pwdf_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

void pwdf_debug_fail_alloc(int after) { g_alloc_budget.store(after < 0 ? -1 : after); }

int64_t pwdf_debug_live_allocs(void) { return g_live.load(); }

void pwdf_destroy(pwdf_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  for (int i = 0; i < kAux; ++i)
    if (c->aux[i]) (void)hipStreamSynchronize(c->aux[i]);
  if (c->cap) (void)hipStreamSynchronize(c->cap);
  drop_graph(c);
  for (hipEvent_t e : c->prof_pool) (void)hipEventDestroy(e);
  for (int i = 0; i < kAux; ++i) {
    if (c->aux[i]) (void)hipStreamDestroy(c->aux[i]);
    if (c->ev_join[i]) (void)hipEventDestroy(c->ev_join[i]);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  free_device(c);
  delete c;
}

}  // extern "C"
