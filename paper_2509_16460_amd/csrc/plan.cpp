// Host plan of libpwdf (see plan.h).
//
// Passages: section "Long-range contributions" (what is computed per pair),
// section "Integral screening" (pair list), appendix "Cartesian coordinates and
// relative coordinates" (A, B, relative coordinates), appendix "Expansion of
// angular prefactor in relative coordinate" (multinomial transform of
// G_x^lx G_y^ly G_z^lz into relative monomials), eq. "FT for D" / "FT of J"
// (phase tables).
#include "plan.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <map>
#include <tuple>

namespace pwdf {

namespace {

constexpr double kPi = 3.14159265358979323846;

double dfact(int n) {
  double r = 1.0;
  for (; n > 1; n -= 2) r *= n;
  return r;
}

double gto_norm(int l, double a) {
  return std::pow(2.0 * a / kPi, 0.75) * std::pow(4.0 * a, 0.5 * l) / std::sqrt(dfact(2 * l - 1));
}

bool lex_nonneg(const std::array<int, 3> &m) {
  for (int i = 0; i < 3; ++i) {
    if (m[i] > 0) return true;
    if (m[i] < 0) return false;
  }
  return true;  // m == 0
}

// |G|^2 for Miller indices n in the original axes, as sum of squared Cartesian components.
double g2_of(const Plan &p, const int n[3]) {
  double s = 0.0;
  for (int c = 0; c < 3; ++c) {
    double g = p.B[c][0] * n[0] + p.B[c][1] * n[1] + p.B[c][2] * n[2];
    s += g * g;
  }
  return s;
}

// Index of a monomial (e0, e1, e2) of degree d in descending lexicographic order.
int mono_index(int e0, int e1, int e2) {
  int d = e0 + e1 + e2;
  // components with first exponent > e0 come first: sum_{x=e0+1}^{d} (d - x + 1)
  int idx = 0;
  for (int x = d; x > e0; --x) idx += d - x + 1;
  idx += (d - e0) - e1;
  return idx;
}

// ---- per-pair cut radius (section "Integral screening") ----
// McMurchie-Davidson Hermite coefficients of one axis (host), E[i][j][t],
// i <= la, j <= lb, t <= i + j.
void md_host(int la, int lb, double p, double xpa, double xpb, double E[4][4][8]) {
  for (int i = 0; i <= la; ++i)
    for (int j = 0; j <= lb; ++j)
      for (int t = 0; t < 8; ++t) E[i][j][t] = 0.0;
  E[0][0][0] = 1.0;
  const double inv2p = 0.5 / p;
  for (int i = 0; i <= la; ++i)
    for (int j = 0; j <= lb; ++j) {
      if (i == 0 && j == 0) continue;
      for (int t = 0; t <= i + j; ++t) {
        double v;
        if (i > 0) {
          v = xpa * E[i - 1][j][t];
          if (t > 0) v += inv2p * E[i - 1][j][t - 1];
          if (t + 1 <= i - 1 + j) v += (t + 1) * E[i - 1][j][t + 1];
        } else {
          v = xpb * E[i][j - 1][t];
          if (t > 0) v += inv2p * E[i][j - 1][t - 1];
          if (t + 1 <= i + j - 1) v += (t + 1) * E[i][j - 1][t + 1];
        }
        E[i][j][t] = v;
      }
    }
}

// Screening objective of one primitive pair at |G| = G:
//   eps(G) = 8 pi eta G (4 pi / G^2) e^{-G^2/4w^2} |F|_inf(G),  eta = [1/p + 1/w^2]^-1,
// |F|_inf the largest modulus over the shell pair's Cartesian components of the
// pair transform with G along x, y or z: with the Hermite expansion
//   |F_ij(G e_d)| = pref K (pi/p)^{3/2} e^{-G^2/4p} |sum_t E^d_{i_d j_d t} (-iG)^t|
//                   prod_{x != d} |E^x_{i_x j_x 0}|.
struct CutPair {
  int la, lb;
  double p, pref, K;
  double E[3][4][4][8];
};

double cut_objective(const CutPair &c, double omega, double G) {
  double fmax = 0.0;
  const double base = c.pref * c.K * std::pow(kPi / c.p, 1.5) * std::exp(-G * G / (4.0 * c.p));
  for (int ia = 0; ia < ncart(c.la); ++ia)
    for (int ib = 0; ib < ncart(c.lb); ++ib) {
      int a[3], b[3];
      // components in descending lexicographic order
      {
        int n = 0;
        for (int x = c.la; x >= 0; --x)
          for (int y = c.la - x; y >= 0; --y, ++n)
            if (n == ia) a[0] = x, a[1] = y, a[2] = c.la - x - y;
        n = 0;
        for (int x = c.lb; x >= 0; --x)
          for (int y = c.lb - x; y >= 0; --y, ++n)
            if (n == ib) b[0] = x, b[1] = y, b[2] = c.lb - x - y;
      }
      for (int d = 0; d < 3; ++d) {
        double re = 0.0, im = 0.0, gp = 1.0;  // sum_t E_t (-iG)^t
        for (int t = 0; t <= a[d] + b[d]; ++t) {
          const double e = c.E[d][a[d]][b[d]][t] * gp;
          switch (t & 3) {
            case 0: re += e; break;
            case 1: im -= e; break;
            case 2: re -= e; break;
            default: im += e; break;
          }
          gp *= G;
        }
        double f = std::sqrt(re * re + im * im);
        for (int x = 0; x < 3; ++x)
          if (x != d) f *= std::fabs(c.E[x][a[x]][b[x]][0]);
        fmax = std::max(fmax, f);
      }
    }
  const double eta = 1.0 / (1.0 / c.p + 1.0 / (omega * omega));
  return 8.0 * kPi * eta * G * (4.0 * kPi / (G * G)) * std::exp(-G * G / (4.0 * omega * omega)) * base * fmax;
}

// Cut radius: from the global cutoff downwards in 256 equal steps to the first G
// where the objective reaches eps_G, then 60 bisection steps on that step; the
// bracket's upper end (the global cutoff if the objective reaches eps_G there).
double cut_radius(const CutPair &c, double omega, double eps_G) {
  const double gglob = 2.0 * omega * std::sqrt(-std::log(eps_G));
  if (cut_objective(c, omega, gglob) >= eps_G) return gglob;
  double hi = gglob, lo = 0.0;
  for (int k = 1; k < 256; ++k) {
    const double G = gglob * (1.0 - k / 256.0);
    if (cut_objective(c, omega, G) >= eps_G) {
      lo = G;
      break;
    }
    hi = G;
  }
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid > 0.0 && cut_objective(c, omega, mid) >= eps_G)
      lo = mid;
    else
      hi = mid;
  }
  return hi;
}

}  // namespace

static void head_points(Plan &p);

// GPW grid and lists of the DD pairs (see Plan::gN).  The ball of a pair density
// is cut at e^{-p r^2} = e^{-50}: with its polynomial factor of degree <= 6 the
// dropped tail stays below ~1e-15 of the pair's values.  Returns a reason when
// the grid work (image boxes x their grid points, collocation and integration
// alike) would exceed kGpwMaxWork: GPW pays off when the cell is large against
// the diffuse Gaussians; for a small cell the analytic route is the one to use.
constexpr double kGpwMaxWork = 3e9;
constexpr int kGpwItems = 2048;

static std::string build_gpw(Plan &p) {
  for (int i = 0; i < 3; ++i) p.gM[i] = 0;
  for (size_t s = 0; s < p.slot_miller.size() / 3; ++s)
    for (int i = 0; i < 3; ++i) p.gM[i] = std::max(p.gM[i], std::abs(p.slot_miller[3 * s + i]));
  for (int i = 0; i < 3; ++i) {
    p.gN[i] = 2 * (int)std::ceil(1.25 * p.gM[i]) + 1;
    p.gtiles[i] = (p.gN[i] + 7) / 8;
  }
  const int ndd = (int)p.dd_q.size();
  p.gP.assign(4 * (size_t)ndd, 0.0);
  p.gimg.clear();
  p.gimg_box.clear();
  p.gimg_off.assign(ndd + 1, 0);
  double work = 0.0;
  double blen[3];
  for (int i = 0; i < 3; ++i)
    blen[i] = std::sqrt(p.B[0][i] * p.B[0][i] + p.B[1][i] * p.B[1][i] + p.B[2][i] * p.B[2][i]);
  for (int k = 0; k < ndd; ++k) {
    const int q = p.dd_q[k];
    const BlockRec &br = p.blocks[p.dd_blk[k]];
    const PairAux &x = p.aux[q];
    const double *RA = &p.in.xyz[3 * p.in.sh_atom[br.sa]];
    double P[3], f[3], rf[3];
    for (int c = 0; c < 3; ++c) P[c] = RA[c] + x.xpa[c];
    const double rc2 = 50.0 / x.p, rc = std::sqrt(rc2);
    for (int c = 0; c < 3; ++c) p.gP[4 * k + c] = P[c];
    p.gP[4 * k + 3] = rc2;
    for (int i = 0; i < 3; ++i) {
      f[i] = (p.B[0][i] * P[0] + p.B[1][i] * P[1] + p.B[2][i] * P[2]) / (2.0 * kPi);
      rf[i] = rc * blen[i] / (2.0 * kPi);  // fractional half-width of the ball along a_i
    }
    int mlo[3], mhi[3];
    for (int i = 0; i < 3; ++i) {
      mlo[i] = (int)std::ceil(-rf[i] - f[i]);
      mhi[i] = (int)std::floor(1.0 + rf[i] - f[i]);
    }
    for (int m0 = mlo[0]; m0 <= mhi[0]; ++m0)
      for (int m1 = mlo[1]; m1 <= mhi[1]; ++m1)
        for (int m2 = mlo[2]; m2 <= mhi[2]; ++m2) {
          const int m[3] = {m0, m1, m2};
          int box[6];
          bool empty = false;
          for (int i = 0; i < 3; ++i) {
            const double c0 = f[i] + m[i];
            box[2 * i] = std::max(0, (int)std::ceil((c0 - rf[i]) * p.gN[i]));
            box[2 * i + 1] = std::min(p.gN[i] - 1, (int)std::floor((c0 + rf[i]) * p.gN[i]));
            empty = empty || box[2 * i] > box[2 * i + 1];
          }
          if (empty) continue;
          work += (double)(box[1] - box[0] + 1) * (box[3] - box[2] + 1) * (box[5] - box[4] + 1);
          if (work > kGpwMaxWork) {
            char msg[256];
            std::snprintf(msg, sizeof msg,
                          "unsupported: the GPW route of the DD pairs would evaluate more than %.0e grid points "
                          "(diffuse Gaussians much wider than the cell); use the analytic route (dd_gpw = 0)",
                          kGpwMaxWork);
            return msg;
          }
          p.gimg.insert(p.gimg.end(), {k, m0, m1, m2});
          p.gimg_box.insert(p.gimg_box.end(), box, box + 6);
        }
    p.gimg_off[k + 1] = (int)(p.gimg.size() / 4);
  }
  // tiles of 8^3 grid points: the image entries whose box meets each tile
  const int nt = p.gtiles[0] * p.gtiles[1] * p.gtiles[2];
  std::vector<std::vector<int>> per(nt);
  const int ne = (int)(p.gimg.size() / 4);
  for (int e = 0; e < ne; ++e) {
    const int *b = &p.gimg_box[6 * (size_t)e];
    for (int t2 = b[4] / 8; t2 <= b[5] / 8; ++t2)
      for (int t1 = b[2] / 8; t1 <= b[3] / 8; ++t1)
        for (int t0 = b[0] / 8; t0 <= b[1] / 8; ++t0) per[(t2 * p.gtiles[1] + t1) * p.gtiles[0] + t0].push_back(e);
  }
  p.gtile_off.assign(nt + 1, 0);
  p.gtile_ent.clear();
  for (int t = 0; t < nt; ++t) {
    p.gtile_off[t] = (int)p.gtile_ent.size();
    p.gtile_ent.insert(p.gtile_ent.end(), per[t].begin(), per[t].end());
  }
  p.gtile_off[nt] = (int)p.gtile_ent.size();
  // about kGpwItems work items over the whole grid, at least 32 entries each
  p.glen = (int)std::max<int64_t>(32, ((int64_t)p.gtile_ent.size() + kGpwItems - 1) / kGpwItems);
  p.gitem.clear();
  p.gitem_off.assign(nt + 1, 0);
  for (int t = 0; t < nt; ++t) {
    p.gitem_off[t] = (int)(p.gitem.size() / 3);
    int a = p.gtile_off[t];
    do {
      const int b = std::min(p.gtile_off[t + 1], a + p.glen);
      p.gitem.insert(p.gitem.end(), {t, a, b});
      a = b;
    } while (a < p.gtile_off[t + 1]);
  }
  p.gitem_off[nt] = (int)(p.gitem.size() / 3);
  return std::string();
}

void build_segments(Plan &p, int seg_len) {
  p.seg_len = seg_len;
  p.segs.clear();
  p.slot_v.clear();
  p.slot_vf.clear();
  p.slot_miller.clear();
  p.valid_slots.clear();
  p.pts.clear();
  const double gcut2 = 4.0 * p.in.omega * p.in.omega * (-std::log(p.in.eps_G));
  const double gcut = std::sqrt(gcut2);
  int nmax[3];
  for (int i = 0; i < 3; ++i) {
    double alen = std::sqrt(p.A[0][i] * p.A[0][i] + p.A[1][i] * p.A[1][i] + p.A[2][i] * p.A[2][i]);
    nmax[i] = (int)std::floor(gcut * alen / (2.0 * kPi)) + 1;
  }
  const int u = p.ax[0], v = p.ax[1], w = p.ax[2];
  const double w4 = 4.0 * p.in.omega * p.in.omega;
  // lines of the half space: (nw > 0) or (nw = 0, nv > 0) or (0, 0, nu > 0), with
  // their n_u range inside the cutoff sphere and their smallest |G|^2
  struct Line {
    double g2min;
    int nw, nv, lo, hi;
  };
  std::vector<Line> lines;
  for (int nw = 0; nw <= nmax[w]; ++nw)
    for (int nv = -nmax[v]; nv <= nmax[v]; ++nv) {
      if (nw == 0 && nv < 0) continue;
      int lo = 1 << 30, hi = -(1 << 30);
      double gmin = 1e300;
      for (int nu = -nmax[u]; nu <= nmax[u]; ++nu) {
        if (nw == 0 && nv == 0 && nu <= 0) continue;
        int n[3];
        n[u] = nu;
        n[v] = nv;
        n[w] = nw;
        double g2 = g2_of(p, n);
        if (g2 > 0.0 && g2 <= gcut2) {
          lo = std::min(lo, nu);
          hi = std::max(hi, nu);
          gmin = std::min(gmin, g2);
        }
      }
      if (lo <= hi) lines.push_back({gmin, nw, nv, lo, hi});
    }
  // lines ordered by their smallest |G| (segments of one line stay adjacent), so
  // that a group of segments or points spans a narrow range of |G|: pairs whose
  // own cut radius is smaller skip whole groups (section "Integral screening")
  std::stable_sort(lines.begin(), lines.end(), [](const Line &a, const Line &b) {
    return std::tie(a.g2min, a.nw, a.nv) < std::tie(b.g2min, b.nw, b.nv);
  });
  int64_t count = 0;
  for (const Line &ln : lines) {
    const int nv = ln.nv, nw = ln.nw;
    for (int nu0 = ln.lo; nu0 <= ln.hi; nu0 += seg_len) {
      SegDesc sd;
      sd.nu0 = nu0;
      sd.nv = nv;
      sd.nw = nw;
      sd.cnt = std::min(seg_len, ln.hi - nu0 + 1);
      double b = p.M[u][v] * nv + p.M[u][w] * nw;
      double c = p.M[v][v] * nv * nv + 2.0 * p.M[v][w] * nv * nw + p.M[w][w] * nw * nw;
      sd.gq0 = p.M[u][u] * nu0 * (double)nu0 + 2.0 * b * nu0 + c;
      sd.dg0 = p.M[u][u] * (2.0 * nu0 + 1.0) + 2.0 * b;
      sd.g2min = 1e300;
      sd.pad = 0.0;
      int sidx = (int)p.segs.size();
      for (int s = 0; s < seg_len; ++s) {
        int n[3] = {0, 0, 0};
        double vg = 0.0, vf = 0.0;
        if (s < sd.cnt) {
          n[u] = nu0 + s;
          n[v] = nv;
          n[w] = nw;
          double g2 = g2_of(p, n);
          vg = 4.0 * kPi * std::exp(-g2 / w4) / g2;
          vf = 4.0 * kPi / g2;
          sd.g2min = std::min(sd.g2min, g2);
          p.valid_slots.push_back(sidx * seg_len + s);
          p.pts.push_back({g2, nu0 + s, nv, nw, sidx * seg_len + s});
          ++count;
        }
        p.slot_v.push_back(vg);
        p.slot_vf.push_back(vf);
        for (int c3 = 0; c3 < 3; ++c3) p.slot_miller.push_back(n[c3]);
      }
      p.segs.push_back(sd);
    }
  }
  p.nG_full = 2 * count;
  // The point list in order of |G|^2 (ties in walk order): a run of consecutive
  // points spans a narrow shell, so the per-pair cuts skip whole K-steps and
  // tiles of the point-wise kernels; v(G) decreases with |G|, so the head (v(G) >=
  // kHeadWeight max v) is a prefix.
  std::stable_sort(p.pts.begin(), p.pts.end(), [](const GPoint &a, const GPoint &b) { return a.g2 < b.g2; });
  head_points(p);
}

// The head: the prefix of the |G|-ordered points with v(G) >= head_weight max v.
static void head_points(Plan &p) {
  const double vmax = p.pts.empty() ? 0.0 : p.slot_v[p.pts[0].slot];
  p.npts_head = 0;
  while (p.npts_head < (int)p.pts.size() && p.slot_v[p.pts[p.npts_head].slot] >= p.head_weight * vmax)
    ++p.npts_head;
  p.head_g2 = p.npts_head > 0 ? p.pts[p.npts_head - 1].g2 : 0.0;
}

// Head points within each pair's cut, per class L and in total.
static void head_pair_counts(Plan &p) {
  std::vector<double> hg2;
  for (int i = 0; i < p.npts_head; ++i) hg2.push_back(p.pts[i].g2);
  std::sort(hg2.begin(), hg2.end());
  p.pairG_head = 0.0;
  for (int L = 0; L <= kMaxLsum; ++L) {
    p.pairG_head_L[L] = 0.0;
    for (int q = p.L_p0[L]; q < p.L_p1[L]; ++q)
      p.pairG_head_L[L] += (double)(std::upper_bound(hg2.begin(), hg2.end(), p.hot[q].gc2) - hg2.begin());
    p.pairG_head += p.pairG_head_L[L];
  }
}

void set_head_weight(Plan &p, double weight) {
  p.head_weight = weight;
  head_points(p);
  head_pair_counts(p);
}

std::string build_plan(const PlanInput &in, int seg_len, Plan &p) {
  p.in = in;
  char msg[256];
  // ---- validation
  if (in.natm < 1) return "natm must be >= 1";
  if (in.nshell < 1) return "nshell must be >= 1";
  if (!(in.omega > 0.0) || !std::isfinite(in.omega)) return "omega must be finite and > 0";
  if (!(in.eps_pair > 0.0 && in.eps_pair < 1.0)) return "eps_pair must be in (0,1)";
  if (!(in.eps_G > 0.0 && in.eps_G < 1.0)) return "eps_G must be in (0,1)";
  for (int i = 0; i < 3; ++i)
    if (in.kmesh[i] < 1) return "kmesh entries must be >= 1";
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(in.lattice[i])) return "lattice is not finite";
  for (double x : in.xyz)
    if (!std::isfinite(x)) return "xyz is not finite";
  int nprim_tot = 0;
  for (int s = 0; s < in.nshell; ++s) {
    if (in.sh_l[s] < 0 || in.sh_l[s] > kMaxL) {
      std::snprintf(msg, sizeof msg, "shell %d: l=%d outside 0..%d", s, in.sh_l[s], kMaxL);
      return msg;
    }
    if (in.sh_atom[s] < 0 || in.sh_atom[s] >= in.natm) {
      std::snprintf(msg, sizeof msg, "shell %d: atom index %d out of range", s, in.sh_atom[s]);
      return msg;
    }
    if (in.sh_nprim[s] < 1) return "shell_nprim must be >= 1";
    nprim_tot += in.sh_nprim[s];
  }
  if ((int)in.exps.size() != nprim_tot || (int)in.coefs.size() != nprim_tot) return "primitive arrays size mismatch";
  for (int i = 0; i < nprim_tot; ++i) {
    if (!(in.exps[i] > 0.0) || !std::isfinite(in.exps[i])) return "exponents must be finite and > 0";
    if (!std::isfinite(in.coefs[i])) return "coefficients must be finite";
  }

  // ---- geometry
  for (int i = 0; i < 3; ++i)
    for (int c = 0; c < 3; ++c) p.A[c][i] = in.lattice[3 * i + c];
  const double(*A)[3] = p.A;
  double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
               A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  double scale = 1.0;
  for (int i = 0; i < 9; ++i) scale = std::max(scale, std::fabs(in.lattice[i]));
  if (!(std::fabs(det) > 1e-10 * scale * scale * scale)) return "lattice is singular";
  p.vol = std::fabs(det);
  double inv[3][3];
  inv[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
  inv[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
  inv[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
  inv[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
  inv[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
  inv[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
  inv[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
  inv[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
  inv[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < 3; ++i) p.B[c][i] = 2.0 * kPi * inv[i][c];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) p.M[i][j] = p.B[0][i] * p.B[0][j] + p.B[1][i] * p.B[1][j] + p.B[2][i] * p.B[2][j];
  // line axis: the longest index range |a_i| (most G per line)
  {
    double len[3];
    for (int i = 0; i < 3; ++i) len[i] = std::sqrt(A[0][i] * A[0][i] + A[1][i] * A[1][i] + A[2][i] * A[2][i]);
    int u = 0;
    for (int i = 1; i < 3; ++i)
      if (len[i] > len[u] * (1 + 1e-12)) u = i;
    p.ax[0] = u;
    p.ax[1] = (u + 1) % 3 < (u + 2) % 3 ? (u + 1) % 3 : (u + 2) % 3;
    p.ax[2] = 3 - u - p.ax[1];
  }

  // ---- basis offsets
  p.sh_bf.assign(in.nshell + 1, 0);
  p.sh_pr.assign(in.nshell + 1, 0);
  for (int s = 0; s < in.nshell; ++s) {
    p.sh_bf[s + 1] = p.sh_bf[s] + ncart(in.sh_l[s]);
    p.sh_pr[s + 1] = p.sh_pr[s] + in.sh_nprim[s];
  }
  p.nbf = p.sh_bf[in.nshell];
  p.nk = in.kmesh[0] * in.kmesh[1] * in.kmesh[2];
  p.bf_shell.resize(p.nbf);
  p.bf_comp.resize(p.nbf);
  for (int s = 0; s < in.nshell; ++s)
    for (int c = 0; c < ncart(in.sh_l[s]); ++c) {
      p.bf_shell[p.sh_bf[s] + c] = s;
      p.bf_comp[p.sh_bf[s] + c] = c;
    }

  build_segments(p, seg_len);
  if (p.valid_slots.empty()) return "the G set is empty (increase omega or decrease eps_G)";

  // ---- unique screened primitive pairs, grouped into (sa, sb, m) blocks
  struct RawPair {
    int ia, ib;
  };
  struct RawBlock {
    int L, la, sa, sb;
    std::array<int, 3> m;
    std::vector<RawPair> prims;
  };
  std::vector<RawBlock> raw;
  const double lneps = -std::log(in.eps_pair);
  for (int sa = 0; sa < in.nshell; ++sa)
    for (int sb = 0; sb < in.nshell; ++sb) {
      int la = in.sh_l[sa], lb = in.sh_l[sb];
      // one representative of (a,b,L) ~ (b,a,-L): la > lb, or la == lb and sa <= sb
      if (la < lb || (la == lb && sa > sb)) continue;
      const double *RA = &in.xyz[3 * in.sh_atom[sa]];
      const double *RB = &in.xyz[3 * in.sh_atom[sb]];
      double d[3] = {RA[0] - RB[0], RA[1] - RB[1], RA[2] - RB[2]};
      std::map<std::array<int, 3>, std::vector<RawPair>> bym;
      for (int ia = p.sh_pr[sa]; ia < p.sh_pr[sa + 1]; ++ia)
        for (int ib = p.sh_pr[sb]; ib < p.sh_pr[sb + 1]; ++ib) {
          double aa = in.exps[ia], ab = in.exps[ib];
          double mu = aa * ab / (aa + ab);
          double R = std::sqrt(lneps / mu);
          if (in.r_max > 0 && in.r_max < R) R = in.r_max;
          int lo[3], hi[3];
          for (int i = 0; i < 3; ++i) {
            double bd = p.B[0][i] * d[0] + p.B[1][i] * d[1] + p.B[2][i] * d[2];
            double bn = std::sqrt(p.B[0][i] * p.B[0][i] + p.B[1][i] * p.B[1][i] + p.B[2][i] * p.B[2][i]);
            lo[i] = (int)std::floor((bd - bn * R) / (2.0 * kPi)) - 1;
            hi[i] = (int)std::ceil((bd + bn * R) / (2.0 * kPi)) + 1;
          }
          for (int m0 = lo[0]; m0 <= hi[0]; ++m0)
            for (int m1 = lo[1]; m1 <= hi[1]; ++m1)
              for (int m2 = lo[2]; m2 <= hi[2]; ++m2) {
                std::array<int, 3> m = {m0, m1, m2};
                if (sa == sb && !lex_nonneg(m)) continue;
                double r2 = 0.0;
                for (int c = 0; c < 3; ++c) {
                  double L = A[c][0] * m0 + A[c][1] * m1 + A[c][2] * m2;
                  double x = d[c] - L;
                  r2 += x * x;
                }
                if (!(std::exp(-mu * r2) >= in.eps_pair)) continue;
                if (in.r_max > 0 && std::sqrt(r2) > in.r_max) continue;
                bym[m].push_back({ia, ib});
              }
        }
      for (auto &kv : bym) raw.push_back({la + lb, la, sa, sb, kv.first, std::move(kv.second)});
    }
  if (raw.empty()) return "no pair survives screening";
  std::stable_sort(raw.begin(), raw.end(), [](const RawBlock &x, const RawBlock &y) {
    return std::tie(x.L, x.la, x.sa, x.sb, x.m) < std::tie(y.L, y.la, y.sa, y.sb, y.m);
  });

  std::map<std::array<int, 3>, int> img_index;
  p.blocks.clear();
  p.hot.clear();
  p.aux.clear();
  for (int c = 0; c < 16; ++c) p.cls_b0[c] = p.cls_b1[c] = 0;
  for (int L = 0; L <= kMaxLsum; ++L) p.L_p0[L] = p.L_p1[L] = 0;
  int64_t eoff = 0;
  for (const RawBlock &rb : raw) {
    auto it = img_index.find(rb.m);
    int img;
    if (it == img_index.end()) {
      img = (int)p.imgs.size();
      img_index[rb.m] = img;
      p.imgs.push_back(rb.m);
    } else {
      img = it->second;
    }
    BlockRec br;
    br.sa = rb.sa;
    br.sb = rb.sb;
    br.img = img;
    br.p0 = (int)p.hot.size();
    br.bfa = p.sh_bf[rb.sa];
    br.bfb = p.sh_bf[rb.sb];
    bool diag = (rb.sa == rb.sb) && rb.m[0] == 0 && rb.m[1] == 0 && rb.m[2] == 0;
    br.w2 = diag ? 0 : 1;
    br.eoff = eoff;
    int la = in.sh_l[rb.sa], lb = in.sh_l[rb.sb];
    eoff += (int64_t)ncart(la) * ncart(lb);
    const double *RA = &in.xyz[3 * in.sh_atom[rb.sa]];
    const double *RB0 = &in.xyz[3 * in.sh_atom[rb.sb]];
    double RB[3];
    for (int c = 0; c < 3; ++c) RB[c] = RB0[c] + A[c][0] * rb.m[0] + A[c][1] * rb.m[1] + A[c][2] * rb.m[2];
    for (const RawPair &pr : rb.prims) {
      double aa = in.exps[pr.ia], ab = in.exps[pr.ib];
      double pp = aa + ab;
      double P[3], r2 = 0.0;
      for (int c = 0; c < 3; ++c) {
        P[c] = (aa * RA[c] + ab * RB[c]) / pp;
        r2 += (RA[c] - RB[c]) * (RA[c] - RB[c]);
      }
      double K = std::exp(-aa * ab / pp * r2);
      double C = in.coefs[pr.ia] * in.coefs[pr.ib] * gto_norm(la, aa) * gto_norm(lb, ab) * K * std::pow(kPi / pp, 1.5);
      PairAux x;
      x.p = pp;
      for (int c = 0; c < 3; ++c) {
        x.xpa[c] = P[c] - RA[c];
        x.xpb[c] = P[c] - RB[c];
      }
      x.pref_rho = (diag ? 1.0 : 2.0) * C / p.vol;
      x.pref_j = 2.0 * C;
      x.alpha_a = aa;
      x.alpha_b = ab;
      x.w = diag ? 1.0 : 2.0;
      x.pad = 0.0;
      PairHot h;
      double f[3];
      for (int i = 0; i < 3; ++i) {
        double t = (p.B[0][i] * P[0] + p.B[1][i] * P[1] + p.B[2][i] * P[2]) / (2.0 * kPi);
        f[i] = t - std::nearbyint(t);
      }
      h.inv4p = 0.25 / pp;
      h.fu = f[p.ax[0]];
      h.fv = f[p.ax[1]];
      h.fw = f[p.ax[2]];
      h.cu = std::cos(2.0 * kPi * h.fu);
      h.su = -std::sin(2.0 * kPi * h.fu);
      h.q = std::exp(-p.M[p.ax[0]][p.ax[0]] / (2.0 * pp));
      h.gc2 = 1e300;  // set per block below when per-pair cuts are on
      p.hot.push_back(h);
      p.aux.push_back(x);
    }
    br.p1 = (int)p.hot.size();
    // per-pair cut: the block's most compact primitive pair (largest p, the first
    // of equal ones) sets the cut radius of all its primitive pairs, as the paper
    // does for a contracted shell pair (section "Integral screening")
    if (in.pair_gcut && br.p1 > br.p0) {
      int best = br.p0;
      for (int q = br.p0 + 1; q < br.p1; ++q)
        if (p.aux[q].p > p.aux[best].p) best = q;
      const RawPair &pr = rb.prims[best - br.p0];
      CutPair cp;
      cp.la = la;
      cp.lb = lb;
      cp.p = p.aux[best].p;
      cp.pref = std::fabs(in.coefs[pr.ia] * in.coefs[pr.ib]) * gto_norm(la, in.exps[pr.ia]) * gto_norm(lb, in.exps[pr.ib]);
      double r2 = 0.0;
      for (int c = 0; c < 3; ++c) r2 += (RA[c] - RB[c]) * (RA[c] - RB[c]);
      cp.K = std::exp(-in.exps[pr.ia] * in.exps[pr.ib] / cp.p * r2);
      for (int x = 0; x < 3; ++x) md_host(la, lb, cp.p, p.aux[best].xpa[x], p.aux[best].xpb[x], cp.E[x]);
      const double rc = cut_radius(cp, in.omega, in.eps_G);
      for (int q = br.p0; q < br.p1; ++q) p.hot[q].gc2 = rc * rc;
    }
    p.blocks.push_back(br);
  }
  p.nelem = eoff;
  // Compact/diffuse classification (section "Density classification: compact
  // and diffuse"; alpha_cut = w^2/2 by eq. "cd cutoff" is the caller's choice):
  // a primitive pair whose two exponents both lie below alpha_cut is a DD pair.
  // Its gc2 of -1 takes it out of the compact pairs' pair-G passes; the DD
  // kernels evaluate it over the whole G set with the full-range potential.
  p.dd_q.clear();
  p.dd_L.clear();
  p.dd_of.assign(p.hot.size(), -1);
  p.dd_blk.clear();
  if (in.alpha_cut > 0.0) {
    for (size_t bi = 0; bi < p.blocks.size(); ++bi) {
      const BlockRec &br = p.blocks[bi];
      const int L = in.sh_l[br.sa] + in.sh_l[br.sb];
      for (int q = br.p0; q < br.p1; ++q)
        if (p.aux[q].alpha_a < in.alpha_cut && p.aux[q].alpha_b < in.alpha_cut) {
          p.dd_of[q] = (int)p.dd_q.size();
          p.dd_q.push_back(q);
          p.dd_L.push_back(L);
          p.dd_blk.push_back((int)bi);
          p.hot[q].gc2 = -1.0;
        }
    }
  }
  if (in.dd_gpw && !p.dd_q.empty()) {
    const std::string why = build_gpw(p);
    if (!why.empty()) return why;
  }
  // Pair-G work inside the cuts: for each pair and G line (fixed n_v, n_w) the
  // n_u with |G(n_u)|^2 = M_uu n_u^2 + 2 b n_u + c <= gc2 lie between the roots
  // of the quadratic (eq. "G-space root finding"), clipped to the line's range.
  {
    struct LineQ {
      double b, c;
      int lo, hi;
    };
    std::vector<LineQ> lq;
    const int u = p.ax[0], v = p.ax[1], w = p.ax[2];
    const double muu = p.M[u][u];
    for (size_t i = 0; i < p.segs.size(); ++i) {
      const SegDesc &sd = p.segs[i];
      if (i > 0 && p.segs[i - 1].nv == sd.nv && p.segs[i - 1].nw == sd.nw) {
        lq.back().hi = sd.nu0 + sd.cnt - 1;
        continue;
      }
      lq.push_back({p.M[u][v] * sd.nv + p.M[u][w] * sd.nw,
                    p.M[v][v] * sd.nv * (double)sd.nv + 2.0 * p.M[v][w] * sd.nv * sd.nw + p.M[w][w] * sd.nw * (double)sd.nw,
                    sd.nu0, sd.nu0 + sd.cnt - 1});
    }
    const double gcut2 = 4.0 * in.omega * in.omega * (-std::log(in.eps_G));
    double last = -1.0, last_cnt = 0.0;
    p.pairG_of.resize(p.hot.size());
    for (size_t q = 0; q < p.hot.size(); ++q) {
      const double gc2 = std::min(p.hot[q].gc2, gcut2 * (1.0 + 1e-12));
      if (gc2 != last) {
        last = gc2;
        last_cnt = 0.0;
        for (const LineQ &l : lq) {
          const double disc = l.b * l.b - muu * (l.c - gc2);
          if (disc < 0.0) continue;
          const double sq = std::sqrt(disc);
          const int lo = std::max(l.lo, (int)std::ceil((-l.b - sq) / muu - 1e-12));
          const int hi = std::min(l.hi, (int)std::floor((-l.b + sq) / muu + 1e-12));
          if (hi >= lo) last_cnt += hi - lo + 1;
        }
      }
      p.pairG_of[q] = last_cnt;
    }
  }
  // Bound of the segment-start arguments: |G|^2 / 4p <= Gcut^2 / 4p and the step
  // ratio (|G(n+1)|^2 - |G(n)|^2) / 4p, |.| <= (2 Gcut |b_u| + |b_u|^2) / 4p, over
  // the smallest p.  The starts are evaluated without range handling (exp of
  // arguments up to ~700) and the recurrence multiplies them: a pair so diffuse
  // that these overflow or underflow is rejected rather than summed as inf / 0.
  {
    // (DD pairs excluded: the DD kernels evaluate their factors directly)
    double pmin = 1e300;
    for (size_t q = 0; q < p.aux.size(); ++q)
      if (p.dd_of[q] < 0) pmin = std::min(pmin, p.aux[q].p);
    if (pmin == 1e300) pmin = 1.0;
    const double gcut2 = 4.0 * in.omega * in.omega * (-std::log(in.eps_G));
    const double bu2 = p.M[p.ax[0]][p.ax[0]];
    p.max_start_arg = std::max(gcut2, 2.0 * std::sqrt(gcut2 * bu2) + bu2) / (4.0 * pmin);
    if (p.max_start_arg > 650.0) {
      std::snprintf(msg, sizeof msg,
                    "unsupported: pair exponent sum p = %.3g is too diffuse for the G set (Gcut^2/4p = %.0f > 650); "
                    "raise the smallest exponent or eps_G (a smaller G cutoff)",
                    pmin, p.max_start_arg);
      return msg;
    }
  }
  // class ranges (blocks are sorted by (L, la) so classes are contiguous)
  for (int c = 0; c < 16; ++c) {
    p.cls_b0[c] = 0;
    p.cls_b1[c] = 0;
  }
  {
    int b = 0, nb = (int)p.blocks.size();
    while (b < nb) {
      int la = in.sh_l[p.blocks[b].sa], lb = in.sh_l[p.blocks[b].sb];
      int e = b;
      while (e < nb && in.sh_l[p.blocks[e].sa] == la && in.sh_l[p.blocks[e].sb] == lb) ++e;
      p.cls_b0[la * 4 + lb] = b;
      p.cls_b1[la * 4 + lb] = e;
      b = e;
    }
  }
  for (int L = 0; L <= kMaxLsum; ++L) {
    p.L_p0[L] = p.L_p1[L] = 0;
  }
  {
    int64_t off = 0;
    for (int L = 0; L <= 2 * kMaxL; ++L) {
      int p0 = -1, p1 = -1;
      for (int la = 0; la <= kMaxL; ++la) {
        int lb = L - la;
        if (lb < 0 || lb > la) continue;
        int c = la * 4 + lb;
        if (p.cls_b1[c] <= p.cls_b0[c]) continue;
        int q0 = p.blocks[p.cls_b0[c]].p0, q1 = p.blocks[p.cls_b1[c] - 1].p1;
        p0 = p0 < 0 ? q0 : std::min(p0, q0);
        p1 = p1 < 0 ? q1 : std::max(p1, q1);
      }
      if (p0 < 0) p0 = p1 = 0;
      p.L_p0[L] = p0;
      p.L_p1[L] = p1;
      p.dhat_off[L] = off;
      off += (int64_t)(p1 - p0) * nherm(L);
    }
    p.dhat_off[kMaxLsum] = off;
    p.dhat_size = off;
  }
  p.pairG_cut = 0.0;
  for (int L = 0; L <= kMaxLsum; ++L) {
    p.pairG_L[L] = 0.0;
    for (int q = p.L_p0[L]; q < p.L_p1[L]; ++q) p.pairG_L[L] += p.pairG_of[q];
    p.pairG_cut += p.pairG_L[L];
  }
  head_pair_counts(p);
  {
    std::vector<int> order(p.hot.size());
    for (size_t i = 0; i < p.hot.size(); ++i) order[i] = (int)i;
    for (int L = 0; L <= 2; ++L)  // the classes whose rho pass reuses p-dependent factors
      std::stable_sort(order.begin() + p.L_p0[L], order.begin() + p.L_p1[L],
                       [&](int x, int y) { return p.hot[x].inv4p < p.hot[y].inv4p; });
    p.rho_rank.resize(p.hot.size());
    p.hot_rho.resize(p.hot.size());
    for (size_t r = 0; r < order.size(); ++r) {
      p.rho_rank[order[r]] = (int)r;
      p.hot_rho[r] = p.hot[order[r]];
    }
  }
  {
    // the walk order of the J pass (both forms) and of the FP32-MFMA rho pass:
    // each class by cut radius, largest first (storage order without cuts)
    std::vector<int> order(p.hot.size());
    for (size_t i = 0; i < p.hot.size(); ++i) order[i] = (int)i;
    for (int L = 0; L <= kMaxLsum; ++L)
      std::stable_sort(order.begin() + p.L_p0[L], order.begin() + p.L_p1[L],
                       [&](int x, int y) { return p.hot[x].gc2 > p.hot[y].gc2; });
    p.cut_rank.resize(p.hot.size());
    p.hot_cut.resize(p.hot.size());
    for (size_t r = 0; r < order.size(); ++r) {
      p.cut_rank[order[r]] = (int)r;
      p.hot_cut[r] = p.hot[order[r]];
    }
    // blocks of each (la, lb) class in the same walk (by the rank of their first pair)
    p.blk_cut.resize(p.blocks.size());
    for (size_t b = 0; b < p.blocks.size(); ++b) p.blk_cut[b] = (int)b;
    for (int c = 0; c < 16; ++c)
      std::stable_sort(p.blk_cut.begin() + p.cls_b0[c], p.blk_cut.begin() + p.cls_b1[c],
                       [&](int x, int y) { return p.cut_rank[p.blocks[x].p0] < p.cut_rank[p.blocks[y].p0]; });
  }
  p.elem_blk.resize(p.nelem);
  for (int b = 0; b < (int)p.blocks.size(); ++b) {
    const BlockRec &br = p.blocks[b];
    int n = ncart(in.sh_l[br.sa]) * ncart(in.sh_l[br.sb]);
    for (int e = 0; e < n; ++e) p.elem_blk[br.eoff + e] = b;
  }

  // ---- phase tables
  int nimg = (int)p.imgs.size();
  p.phD.assign((size_t)nimg * p.nk * 2, 0.0);
  p.phJ.assign((size_t)nimg * p.nk * 2, 0.0);
  for (int i = 0; i < nimg; ++i)
    for (int k = 0; k < p.nk; ++k) {
      int km[3];
      km[2] = k % in.kmesh[2];
      km[1] = (k / in.kmesh[2]) % in.kmesh[1];
      km[0] = k / (in.kmesh[2] * in.kmesh[1]);
      // reduce the integer phase exactly before converting: k.L/2pi = sum_i km_i m_i / n_i
      double t = 0.0;
      for (int d = 0; d < 3; ++d) {
        long r = ((long)km[d] * p.imgs[i][d]) % in.kmesh[d];
        t += (double)r / in.kmesh[d];
      }
      t -= std::nearbyint(t);
      double c = std::cos(2.0 * kPi * t), s = std::sin(2.0 * kPi * t);
      size_t o = ((size_t)i * p.nk + k) * 2;
      p.phJ[o] = c;
      p.phJ[o + 1] = s;
      p.phD[o] = c / p.nk;
      p.phD[o + 1] = s / p.nk;
    }

  // ---- J(k) gather lists per ordered shell pair
  {
    int ns = in.nshell;
    std::vector<std::vector<GatherEnt>> lists((size_t)ns * ns);
    for (int b = 0; b < (int)p.blocks.size(); ++b) {
      const BlockRec &br = p.blocks[b];
      lists[(size_t)br.sa * ns + br.sb].push_back({b, br.img, 0, 0});
      if (br.w2) lists[(size_t)br.sb * ns + br.sa].push_back({b, br.img, 1, 0});
    }
    p.sp_off.assign((size_t)ns * ns + 1, 0);
    p.sp_ent.clear();
    for (size_t i = 0; i < lists.size(); ++i) {
      p.sp_off[i] = (int)p.sp_ent.size();
      for (auto &e : lists[i]) p.sp_ent.push_back(e);
    }
    p.sp_off[lists.size()] = (int)p.sp_ent.size();
    // per element lists with integer phase codes
    auto gcd = [](int x, int y) {
      while (y) {
        int t = x % y;
        x = y;
        y = t;
      }
      return x;
    };
    int N = 1;
    for (int i = 0; i < 3; ++i) N = N / gcd(N, in.kmesh[i]) * in.kmesh[i];
    p.phN = N;
    const int T = (in.kmesh[0] + in.kmesh[1] + in.kmesh[2]) * N;
    p.ptab.resize(2 * (size_t)T);
    for (int t = 0; t < T; ++t) {
      int r = t % N;  // exact reduction before the transcendental
      p.ptab[2 * t] = std::cos(2.0 * kPi * r / N);
      p.ptab[2 * t + 1] = std::sin(2.0 * kPi * r / N);
    }
    // class code of image m (sign s = +1) or of -m (s = -1)
    auto code_of = [&](const std::array<int, 3> &m, int s) {
      int c[3];
      for (int d = 0; d < 3; ++d) {
        int n = in.kmesh[d];
        c[d] = ((((s * m[d]) % n) + n) % n) * (N / n);
      }
      return c[0] | (c[1] << 10) | (c[2] << 20);
    };
    const int nbf = p.nbf;
    p.sJ_off.assign((size_t)nbf * nbf + 1, 0);
    p.nD_support = 0;
    p.heavyJ.clear();
    p.lightJ.clear();
    p.sD_el.clear();
    p.sJ_code.clear();
    p.sJ_e0.clear();
    p.eJ.clear();
    p.sD_code.clear();
    p.sD_e0.clear();
    p.eD.clear();
    std::vector<std::pair<int, int>> ents;  // (code, element offset)
    // D side: (element of D(k) read, class code, D(L) offset) of every direct
    // block entry.  The element read is (mu, nu) with the class of m, or, when
    // shell a has more Cartesian components than shell b, the transposed
    // element (nu, mu) with the class of -m (Hermitian D(k):
    // Re e^{ik.m} D_mu,nu(k) = Re e^{-ik.m} D_nu,mu(k)): a row of D(k) then
    // holds ncart(la) consecutive elements of the block instead of ncart(lb),
    // so the lines fetched carry more of the support.
    std::vector<std::array<int, 3>> dtrip;
    // packed layout candidates: (element, class code, D(L) offset, transposed
    // element, its class code), the transposed one taken when shell(mu) > shell(nu)
    std::vector<std::array<int, 5>> ptrip;
    for (int mu = 0; mu < nbf; ++mu)
      for (int nu = 0; nu < nbf; ++nu) {
        size_t e = (size_t)mu * nbf + nu;
        p.sJ_off[e] = (int)p.sJ_code.size();
        int sa = p.bf_shell[mu], sb = p.bf_shell[nu];
        int a = p.bf_comp[mu], b = p.bf_comp[nu];
        const bool dT = ncart(in.sh_l[sa]) > ncart(in.sh_l[sb]);
        ents.clear();
        for (int i = p.sp_off[(size_t)sa * ns + sb]; i < p.sp_off[(size_t)sa * ns + sb + 1]; ++i) {
          const GatherEnt &g = p.sp_ent[i];
          const BlockRec &br = p.blocks[g.blk];
          int ncb = ncart(in.sh_l[br.sb]);
          int64_t joff = br.eoff + (g.tr ? (int64_t)b * ncb + a : (int64_t)a * ncb + b);
          int code = code_of(p.imgs[g.img], g.tr ? -1 : 1);
          ents.push_back({code, (int)joff});
          if (!g.tr) {
            const int codeT = code_of(p.imgs[g.img], -1);
            dtrip.push_back({dT ? nu * nbf + mu : (int)e, dT ? codeT : code, (int)joff});
            ptrip.push_back({(int)e, code, (int)joff, sa > sb ? nu * nbf + mu : -1, codeT});
          }
        }
        std::sort(ents.begin(), ents.end());
        for (size_t i = 0; i < ents.size(); ++i) {
          if (i == 0 || ents[i].first != ents[i - 1].first) {
            p.sJ_code.push_back(ents[i].first);
            p.sJ_e0.push_back((int)p.eJ.size());
          }
          p.eJ.push_back(ents[i].second);
        }
        const int ncls = (int)p.sJ_code.size() - p.sJ_off[e];
        if (ncls > kPhaseLight)
          p.heavyJ.push_back((int)e);
        else if (ncls > 0)
          p.lightJ.push_back((int)e);
      }
    p.sJ_off[(size_t)nbf * nbf] = (int)p.sJ_code.size();
    p.sJ_e0.push_back((int)p.eJ.size());
    // D segments: one per (element read, class), ordered by element
    std::sort(dtrip.begin(), dtrip.end());
    for (size_t i = 0; i < dtrip.size(); ++i) {
      const bool new_el = i == 0 || dtrip[i][0] != dtrip[i - 1][0];
      if (new_el || dtrip[i][1] != dtrip[i - 1][1]) {
        p.sD_el.push_back(dtrip[i][0]);
        p.sD_code.push_back(dtrip[i][1]);
        p.sD_e0.push_back((int)p.eD.size());
      }
      if (new_el) ++p.nD_support;
      p.eD.push_back(dtrip[i][2]);
    }
    p.sD_e0.push_back((int)p.eD.size());
    // packed D segments: element = index in the packed order (lightJ, then heavyJ)
    std::vector<int> pidx((size_t)nbf * nbf, -1);
    int np = 0;
    for (const std::vector<int> *v : {&p.lightJ, &p.heavyJ})
      for (int e : *v) pidx[e] = np++;
    for (auto &t : ptrip) {
      const bool tr = t[3] >= 0 && pidx[t[3]] >= 0;
      t = {pidx[tr ? t[3] : t[0]], tr ? t[4] : t[1], t[2], 0, 0};
      if (t[0] < 0) return "internal: a D(L) entry outside the J(k) support";
    }
    std::sort(ptrip.begin(), ptrip.end());
    p.sDp_el.clear();
    p.sDp_code.clear();
    p.sDp_e0.clear();
    p.eDp.clear();
    p.nDp_support = 0;
    for (size_t i = 0; i < ptrip.size(); ++i) {
      if (i == 0 || ptrip[i][0] != ptrip[i - 1][0]) ++p.nDp_support;
      if (i == 0 || ptrip[i][0] != ptrip[i - 1][0] || ptrip[i][1] != ptrip[i - 1][1]) {
        p.sDp_el.push_back(ptrip[i][0]);
        p.sDp_code.push_back(ptrip[i][1]);
        p.sDp_e0.push_back((int)p.eDp.size());
      }
      p.eDp.push_back(ptrip[i][2]);
    }
    p.sDp_e0.push_back((int)p.eDp.size());
  }

  // ---- Hermite -> relative monomial transform per degree:
  // G_x^tx G_y^ty G_z^tz = sum_k T[t][k] n_u^ku n_v^kv n_w^kw, G_c = sum_j B[c][ax[j]] n_(ax j)
  p.ttab.assign(kTTableSize, 0.0);
  for (int d = 0; d <= kMaxLsum; ++d) {
    int nc = ncart(d);
    int t = 0;
    for (int tx = d; tx >= 0; --tx)
      for (int ty = d - tx; ty >= 0; --ty, ++t) {
        int tz = d - tx - ty;
        // polynomial as map (e0,e1,e2) -> coefficient
        std::map<std::array<int, 3>, double> poly;
        poly[{0, 0, 0}] = 1.0;
        int tc[3] = {tx, ty, tz};
        for (int c = 0; c < 3; ++c)
          for (int r = 0; r < tc[c]; ++r) {
            std::map<std::array<int, 3>, double> np;
            for (auto &kv : poly)
              for (int j = 0; j < 3; ++j) {
                std::array<int, 3> e = kv.first;
                e[j] += 1;
                np[e] += kv.second * p.B[c][p.ax[j]];
              }
            poly.swap(np);
          }
        for (auto &kv : poly) {
          int k = mono_index(kv.first[0], kv.first[1], kv.first[2]);
          p.ttab[tblk_off(d) + t * nc + k] = kv.second;
        }
      }
  }
  return "";
}

}  // namespace pwdf
