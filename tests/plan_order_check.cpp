// Invariants of the pair order the rho pass walks (plan.cpp), checked on the
// host: rho_rank is a permutation that maps every class range [L_p0, L_p1) onto
// itself; hot_rho holds the pair records in that order (bit for bit); the classes
// L <= 2 are sorted by p (1/(4p) ascending) with ties kept in storage order; the
// classes L >= 3 keep storage order.  The D segments of the packed D(k) layout
// read every D(L) entry once, as the dense ones do, from the same element or its
// Hermitian partner with the negated class, always at shell(mu) <= shell(nu), in
// ascending packed order.  Reads the problem as whitespace-separated
// text: lattice (9), natm and xyz, nshell and shell atoms, shell l, shell primitive
// counts, primitive count and exponents, coefficients, kmesh (3), omega, eps_pair,
// eps_G, r_max, and optionally pair_gcut, alpha_cut, dd_gpw.  Prints "pairs <n>
// classes <m> bad <b>" and exits non-zero on a violation.
//
// With a second argument "sweep" it then rebuilds the segments for every segment
// length the tuner can pick (4, 5, 8, 16) and recounts the head of the G set for
// several weights, checking that the valid slots hold the same G vectors each
// time (same count, each Miller index once, padding at (0,0,0) with v = 0) and
// that the head grows with a smaller weight.  Built with the address and
// undefined-behaviour sanitizers, this runs the host planning code over cells with
// per-pair cuts, DD pairs and the GPW lists.
#include <cstdio>
#include <cstring>
#include <fstream>
#include <set>
#include <tuple>
#include <vector>

#include "plan.h"

using namespace pwdf;

int main(int argc, char **argv) {
  if (argc < 2) return 2;
  std::ifstream f(argv[1]);
  PlanInput in;
  for (double &x : in.lattice) f >> x;
  f >> in.natm;
  in.xyz.resize(3 * in.natm);
  for (double &x : in.xyz) f >> x;
  f >> in.nshell;
  in.sh_atom.resize(in.nshell);
  in.sh_l.resize(in.nshell);
  in.sh_nprim.resize(in.nshell);
  for (int &x : in.sh_atom) f >> x;
  for (int &x : in.sh_l) f >> x;
  for (int &x : in.sh_nprim) f >> x;
  int nprim = 0;
  f >> nprim;
  in.exps.resize(nprim);
  in.coefs.resize(nprim);
  for (double &x : in.exps) f >> x;
  for (double &x : in.coefs) f >> x;
  f >> in.kmesh[0] >> in.kmesh[1] >> in.kmesh[2] >> in.omega >> in.eps_pair >> in.eps_G >> in.r_max;
  if (!f) return 2;
  int gcut = 0, gpw = 0;
  double acut = 0.0;
  if (f >> gcut >> acut >> gpw) {
    in.pair_gcut = gcut;
    in.alpha_cut = acut;
    in.dd_gpw = gpw;
  }
  Plan p;
  const std::string err = build_plan(in, 8, p);
  if (!err.empty()) {
    std::printf("plan error: %s\n", err.c_str());
    return 2;
  }
  const int n = (int)p.hot.size();
  long bad = 0;
  if ((int)p.rho_rank.size() != n || (int)p.hot_rho.size() != n) {
    std::printf("pairs %d classes 0 bad 1\n", n);
    return 1;
  }
  std::vector<int> order(n, -1);
  int classes = 0;
  for (int L = 0; L <= kMaxLsum; ++L) {
    const int p0 = p.L_p0[L], p1 = p.L_p1[L];
    if (p1 > p0) ++classes;
    for (int q = p0; q < p1; ++q) {
      const int r = p.rho_rank[q];
      if (r < p0 || r >= p1 || order[r] != -1) {
        bad++;
        continue;
      }
      order[r] = q;
      if (std::memcmp(&p.hot_rho[r], &p.hot[q], sizeof(PairHot)) != 0) bad++;
      if (L >= 3 && r != q) bad++;
    }
    for (int r = p0 + 1; L <= 2 && r < p1; ++r) {
      const double a = p.hot_rho[r - 1].inv4p, b = p.hot_rho[r].inv4p;
      if (a > b) bad++;                                   // sorted by p
      if (a == b && order[r - 1] > order[r]) bad++;       // stable
    }
  }
  for (int r = 0; r < n; ++r)
    if (order[r] < 0) bad++;
  {
    // D(L) entry -> (dense element read, class code), for both layouts
    std::vector<int> pel;
    for (const std::vector<int> *v : {&p.lightJ, &p.heavyJ}) pel.insert(pel.end(), v->begin(), v->end());
    const size_t ne = p.eD.size();
    std::vector<std::pair<int, int>> dn(p.nelem, {-1, -1}), pk(p.nelem, {-1, -1});
    if (p.eDp.size() != ne || p.sDp_e0.size() != p.sDp_el.size() + 1) bad++;
    for (size_t s = 0; s + 1 < p.sD_e0.size(); ++s)
      for (int j = p.sD_e0[s]; j < p.sD_e0[s + 1]; ++j) {
        if (dn[p.eD[j]].first >= 0) bad++;
        dn[p.eD[j]] = {p.sD_el[s], p.sD_code[s]};
      }
    for (size_t s = 0; s + 1 < p.sDp_e0.size(); ++s) {
      const int el = p.sDp_el[s];
      if (el < 0 || el >= (int)pel.size() || (s > 0 && el < p.sDp_el[s - 1])) {
        bad++;
        continue;
      }
      const int e = pel[el];
      if (p.bf_shell[e / p.nbf] > p.bf_shell[e % p.nbf]) bad++;
      for (int j = p.sDp_e0[s]; j < p.sDp_e0[s + 1]; ++j) {
        if (pk[p.eDp[j]].first >= 0) bad++;
        pk[p.eDp[j]] = {e, p.sDp_code[s]};
      }
    }
    const int N = p.phN;
    auto neg = [N](int c) {
      int r = 0;
      for (int i = 0; i < 3; ++i) r |= ((N - ((c >> (10 * i)) & 1023)) % N) << (10 * i);
      return r;
    };
    for (int64_t j = 0; j < p.nelem; ++j) {
      if ((dn[j].first < 0) != (pk[j].first < 0)) {
        bad++;
        continue;
      }
      if (dn[j].first < 0) continue;
      const int a = dn[j].first, b = pk[j].first;
      const int aT = (a % p.nbf) * p.nbf + a / p.nbf;
      if (!((a == b && dn[j].second == pk[j].second) || (aT == b && neg(dn[j].second) == pk[j].second))) bad++;
    }
  }
  if (argc > 2 && std::strcmp(argv[2], "sweep") == 0) {
    std::set<std::tuple<int, int, int>> ref;
    long nvalid = -1;
    for (int seg : {4, 5, 8, 16, 8}) {
      build_segments(p, seg);
      std::set<std::tuple<int, int, int>> got;
      for (int s : p.valid_slots) {
        const int *m = &p.slot_miller[3 * (size_t)s];
        if (!got.insert({m[0], m[1], m[2]}).second) bad++;  // each G once
      }
      std::vector<char> valid(p.nslot(), 0);
      for (int s : p.valid_slots) valid[s] = 1;
      for (int s = 0; s < p.nslot(); ++s)
        if (!valid[s] && (p.slot_v[s] != 0.0 || p.slot_miller[3 * (size_t)s] != 0 ||
                          p.slot_miller[3 * (size_t)s + 1] != 0 || p.slot_miller[3 * (size_t)s + 2] != 0))
          bad++;
      if (nvalid < 0) {
        nvalid = (long)p.valid_slots.size();
        ref = got;
      } else if ((long)p.valid_slots.size() != nvalid || got != ref) {
        bad++;
      }
    }
    int prev = -1;
    for (double w : {1.0, 1.0 / 1024, 1.0 / 65536, 1.0 / 1048576}) {
      set_head_weight(p, w);
      if (p.npts_head < prev || p.npts_head > (int)p.pts.size()) bad++;
      prev = p.npts_head;
    }
    std::printf("sweep: G %ld head %d dd %zu gpw %d x %d x %d\n", nvalid, prev, p.dd_q.size(), p.gN[0], p.gN[1],
                p.gN[2]);
  }
  std::printf("pairs %d classes %d bad %ld\n", n, classes, bad);
  return bad != 0;
}
