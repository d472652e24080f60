/*
 * pwdf_oracle.c -- plain, slow FP64 CPU oracle for the long-range Coulomb matrix
 * of a periodic Gaussian basis (integral-direct planewave density fitting,
 * arXiv 2509.16460).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library; it builds its own reciprocal
 * lattice, G set, pair list and phase factors from the definitions below.
 *
 * What it computes (the plain definition, no blocking, no reordering):
 *   geometry      A = [a1 a2 a3] (columns), Omega = |det A|, B = 2 pi A^-T
 *                 (appendix "Cartesian coordinates and relative coordinates").
 *   G set         {G = B n : 0 < |G|^2 <= Gcut^2}, Gcut = 2 omega sqrt(-ln eps_G);
 *                 G = 0 is excluded (Ewald split, eq. "Ewald J").
 *   pairs         primitive pairs (a in cell 0, b in cell L = A m) kept when
 *                 K = exp(-a_a a_b / p |A - B - L|^2) >= eps_pair (and the
 *                 centre distance <= r_max if r_max > 0); the Gaussian product
 *                 prefactor of eq. "Gaussian product of the radial decay".
 *   D(L)          sum_k w_k e^{ik.L} D(k)  (eq. "FT for D", weights 1/Nk).
 *   pair FT       (mu 0 nu L | G) = int phi_a(r) phi_b(r-L) e^{-iG.r} dr
 *                 (eq. "AFT for pair density"), evaluated per Cartesian axis
 *                 by the binomial Gaussian-product expansion (eq. "Gaussian
 *                 product of angular prefactor") followed by the Hermite-
 *                 polynomial transform of x_P^n e^{-p x_P^2} (eq. "FT of cart
 *                 Gaussians", Hermite appendix).  The transform of x^n
 *                 e^{-p x^2} under e^{-iGx} carries (-i/(2 sqrt p))^n: the
 *                 printed (+i) factor contradicts the e^{-iG.r} kernel of the
 *                 pair-density definition for odd n, and the sign here is the
 *                 one the definition implies.
 *   rho(G)        (1/Omega) sum_pairs D_ab(L) F_abL(G), for every G in the set.
 *   V, J          v(G) = 4 pi e^{-G^2/4w^2} / G^2;
 *                 J_ab(L) = sum_G v(G) rho(-G) F_abL(G)  (long-range contraction
 *                 order: rho(-G), V(-G), J += F(G) V(-G)).
 *   J(k)          sum_L e^{ik.L} J(L)  (eq. "FT of J").
 *   E_J           1/2 sum D(L) J(L) = 1/2 Omega sum_G v rho(G) rho(-G)
 *                 = 1/2 sum_k w_k sum D(k) J(k): all three are returned.
 *   gradient      dE_J/dR_A = Re sum_G v(G) rho(-G) sum_pairs D_ab dF_abL(G)/dR_A
 *                 at fixed D(k), fixed pair list and fixed G set; the centre
 *                 derivative of a Cartesian Gaussian is 2 alpha (l+1 term)
 *                 - l (l-1 term).
 *   pair cuts     optional (pair_gcut = 1; section "Integral screening"): every
 *                 block of pairs (shell a, shell b, image m) sees only the G with
 *                 |G| <= its cut radius, the largest |G| below Gcut where the
 *                 screening objective 8 pi eta G (4 pi/G^2) e^{-G^2/4w^2}
 *                 |F|_inf(G), eta = [1/p + 1/w^2]^-1 (eqs. "AFT screening obj",
 *                 "eta_munu"), of the block's most compact primitive pair still
 *                 reaches eps_G.  Readings (the text leaves them open): |F|_inf
 *                 is the largest modulus over the block's Cartesian components
 *                 with G along x, along y and along z; the radius is found by a
 *                 scan of 256 steps down from Gcut and 60 bisection steps, and
 *                 is the upper end of the final bracket.  Without cuts every
 *                 pair sees the whole G set.
 *   classification optional (alpha_cut > 0; section "Density classification:
 *                 compact and diffuse", eq. "cd cutoff" gives alpha_cut =
 *                 w^2/2): a primitive function is diffuse when its exponent is
 *                 below alpha_cut, and a primitive pair is a diffuse (DD) pair
 *                 when both of its functions are; every other pair is compact
 *                 (CC or CD).  rho = rho_C + rho_D splits by pair class.  When
 *                 both sides of an interaction are compact it keeps the
 *                 long-range kernel; otherwise the interaction is taken in full
 *                 in reciprocal space, v_full(G) = 4 pi / G^2 (G != 0), so the
 *                 two potentials are
 *                   V_C(G) = v(G) rho_C(G) + v_full(G) rho_D(G)   (compact pairs)
 *                   V_D(G) = v_full(G) (rho_C(G) + rho_D(G))       (DD pairs)
 *                 J_ab(L) = sum_G V_class(-G) F_abL(G) with the pair's own
 *                 class, E_J = 1/2 Omega sum_G [rho_C(G) V_C(-G) + rho_D(G)
 *                 V_D(-G)] (the same three routes), and the gradient takes the
 *                 same V.  Readings: a pair whose exponents equal alpha_cut is
 *                 compact; DD pairs see the whole G set even with per-pair
 *                 cuts (the cut objective is the long-range one); the G set
 *                 stays the long-range one (a DD pair density decays as
 *                 e^{-G^2/4p}, p < w^2, faster than the long-range kernel).
 *
 * Conventions: lattice rows are a1,a2,a3; Cartesian components of a shell in
 * descending lexicographic (lx,ly,lz) order; every component of a primitive
 * carries N(l,a) = (2a/pi)^{3/4} (4a)^{l/2} / sqrt((2l-1)!!); k-points
 * k = sum_i (m_i/n_i) b_i, m_i = 0..n_i-1, flattened row-major.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex zd;

#define ORC_PI 3.14159265358979323846
#define ORC_LMAX 5 /* one above the largest supported shell l (4) for derivatives */

/* ------------------------------------------------------------------------- */
/* small helpers                                                              */
/* ------------------------------------------------------------------------- */

static int ncart_of(int l) { return (l + 1) * (l + 2) / 2; }

static void cart_list(int l, int (*c)[3]) {
  int n = 0;
  for (int lx = l; lx >= 0; --lx)
    for (int ly = l - lx; ly >= 0; --ly) {
      c[n][0] = lx;
      c[n][1] = ly;
      c[n][2] = l - lx - ly;
      ++n;
    }
}

static double dfact(int n) {
  double r = 1.0;
  while (n > 1) {
    r *= n;
    n -= 2;
  }
  return r;
}

static double norm_of(int l, double a) {
  return pow(2.0 * a / ORC_PI, 0.75) * pow(4.0 * a, 0.5 * l) / sqrt(dfact(2 * l - 1));
}

static double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

/* A[c][i] = component c of a_i; B = 2 pi A^{-T}; returns Omega. */
static double lattice_setup(const double *lat, double A[3][3], double B[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int c = 0; c < 3; ++c) A[c][i] = lat[3 * i + c];
  double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
               A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
               A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
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
  /* B^T A = 2 pi I  =>  B = 2 pi (A^{-1})^T  =>  B[c][i] = 2 pi inv[i][c] */
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < 3; ++i) B[c][i] = 2.0 * ORC_PI * inv[i][c];
  return fabs(det);
}

/* ------------------------------------------------------------------------- */
/* the pair Fourier transform, one Cartesian axis at a time                   */
/* ------------------------------------------------------------------------- */

/* Physicists' Hermite polynomials by H_n = 2x H_{n-1} - 2(n-1) H_{n-2}. */
static void hermite(int nmax, double x, double *H) {
  H[0] = 1.0;
  if (nmax >= 1) H[1] = 2.0 * x;
  for (int n = 2; n <= nmax; ++n) H[n] = 2.0 * x * H[n - 1] - 2.0 * (n - 1) * H[n - 2];
}

/* M_n(G) = int u^n e^{-p u^2} e^{-iGu} du
 *        = sqrt(pi/p) (-i/(2 sqrt p))^n H_n(G/(2 sqrt p)) e^{-G^2/(4p)}. */
static void hermite_ft(int nmax, double p, double G, zd *M) {
  double H[2 * ORC_LMAX + 2];
  double sp = sqrt(p);
  hermite(nmax, G / (2.0 * sp), H);
  double g = sqrt(ORC_PI / p) * exp(-G * G / (4.0 * p));
  zd fac = 1.0;
  zd step = -I / (2.0 * sp);
  for (int n = 0; n <= nmax; ++n) {
    M[n] = g * fac * H[n];
    fac *= step;
  }
}

/* f[i][j] = int (x-Ax)^i (x-Bx)^j e^{-aa (x-Ax)^2 - ab (x-Bx)^2} e^{-iGx} dx
 * for i <= imax, j <= jmax, through the Gaussian product theorem:
 *   (x-Ax)^i (x-Bx)^j = sum_{i',j'} C(i,i') C(j,j') X_PA^{i-i'} X_PB^{j-j'} x_P^{i'+j'}
 *   e^{-aa x_A^2} e^{-ab x_B^2} = K_x e^{-p x_P^2}
 *   int x_P^n e^{-p x_P^2} e^{-iGx} dx = e^{-iG P} M_n(G). */
static void ft_axis(int imax, int jmax, double aa, double Ax, double ab, double Bx, double G,
                    zd f[ORC_LMAX + 1][ORC_LMAX + 1]) {
  double p = aa + ab;
  double P = (aa * Ax + ab * Bx) / p;
  double XPA = P - Ax, XPB = P - Bx;
  double Kx = exp(-(aa * ab / p) * (Ax - Bx) * (Ax - Bx));
  zd M[2 * ORC_LMAX + 2];
  hermite_ft(imax + jmax, p, G, M);
  zd ph = cos(G * P) - I * sin(G * P);
  for (int i = 0; i <= imax; ++i)
    for (int j = 0; j <= jmax; ++j) {
      zd s = 0.0;
      for (int ii = 0; ii <= i; ++ii)
        for (int jj = 0; jj <= j; ++jj)
          s += binom(i, ii) * binom(j, jj) * pow(XPA, i - ii) * pow(XPB, j - jj) * M[ii + jj];
      f[i][j] = Kx * ph * s;
    }
}

/* ------------------------------------------------------------------------- */
/* problem description and lists                                              */
/* ------------------------------------------------------------------------- */

typedef struct {
  double A[3][3], B[3][3], omega_vol;
  int natm, nshell, nbf, nk;
  const double *xyz;
  const int *sh_atom, *sh_l, *sh_nprim;
  const double *exps, *coefs;
  int *sh_off;  /* first basis function of each shell */
  int *pr_off;  /* first primitive of each shell */
  int kmesh[3];
  double omega, eps_pair, eps_G, r_max;
} orc_sys;

typedef struct {
  int sa, sb, ia, ib; /* shells and absolute primitive indices */
  int m[3];           /* image: L = A m */
  double L[3];
} orc_pair;

typedef struct {
  int n[3];
  double G[3];
  double G2;
} orc_gvec;

static int sys_setup(orc_sys *s, const double *lattice, int natm, const double *xyz, int nshell,
                     const int *shell_atom, const int *shell_l, const int *shell_nprim,
                     const double *exps, const double *coefs, const int *kmesh, double omega,
                     double eps_pair, double eps_G, double r_max) {
  memset(s, 0, sizeof(*s));
  s->omega_vol = lattice_setup(lattice, s->A, s->B);
  if (!(s->omega_vol > 0)) return -1;
  s->natm = natm;
  s->nshell = nshell;
  s->xyz = xyz;
  s->sh_atom = shell_atom;
  s->sh_l = shell_l;
  s->sh_nprim = shell_nprim;
  s->exps = exps;
  s->coefs = coefs;
  s->sh_off = (int *)malloc(sizeof(int) * (nshell + 1));
  s->pr_off = (int *)malloc(sizeof(int) * (nshell + 1));
  s->sh_off[0] = 0;
  s->pr_off[0] = 0;
  for (int i = 0; i < nshell; ++i) {
    if (shell_l[i] < 0 || shell_l[i] > 4) return -1;
    s->sh_off[i + 1] = s->sh_off[i] + ncart_of(shell_l[i]);
    s->pr_off[i + 1] = s->pr_off[i] + shell_nprim[i];
  }
  s->nbf = s->sh_off[nshell];
  for (int i = 0; i < 3; ++i) s->kmesh[i] = kmesh[i];
  s->nk = kmesh[0] * kmesh[1] * kmesh[2];
  s->omega = omega;
  s->eps_pair = eps_pair;
  s->eps_G = eps_G;
  s->r_max = r_max;
  return 0;
}

static void sys_free(orc_sys *s) {
  free(s->sh_off);
  free(s->pr_off);
}

static int cmp_gvec(const void *x, const void *y) {
  const orc_gvec *a = (const orc_gvec *)x, *b = (const orc_gvec *)y;
  int na = a->n[0] * a->n[0] + a->n[1] * a->n[1] + a->n[2] * a->n[2];
  int nb = b->n[0] * b->n[0] + b->n[1] * b->n[1] + b->n[2] * b->n[2];
  if (na != nb) return na < nb ? -1 : 1;
  for (int i = 0; i < 3; ++i)
    if (a->n[i] != b->n[i]) return a->n[i] < b->n[i] ? -1 : 1;
  return 0;
}

/* All G = B n with 0 < |G|^2 <= Gcut^2, sorted by (|n|^2, n). */
static orc_gvec *make_gvecs(const orc_sys *s, int *ng) {
  double gcut2 = 4.0 * s->omega * s->omega * (-log(s->eps_G));
  double gcut = sqrt(gcut2);
  int nmax[3];
  for (int i = 0; i < 3; ++i) {
    double alen = sqrt(s->A[0][i] * s->A[0][i] + s->A[1][i] * s->A[1][i] + s->A[2][i] * s->A[2][i]);
    nmax[i] = (int)floor(gcut * alen / (2.0 * ORC_PI)) + 1;
  }
  size_t cap = (size_t)(2 * nmax[0] + 1) * (2 * nmax[1] + 1) * (2 * nmax[2] + 1);
  orc_gvec *g = (orc_gvec *)malloc(sizeof(orc_gvec) * cap);
  int n = 0;
  for (int n1 = -nmax[0]; n1 <= nmax[0]; ++n1)
    for (int n2 = -nmax[1]; n2 <= nmax[1]; ++n2)
      for (int n3 = -nmax[2]; n3 <= nmax[2]; ++n3) {
        double G[3];
        for (int c = 0; c < 3; ++c) G[c] = s->B[c][0] * n1 + s->B[c][1] * n2 + s->B[c][2] * n3;
        double G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
        if (G2 > 0.0 && G2 <= gcut2) {
          g[n].n[0] = n1;
          g[n].n[1] = n2;
          g[n].n[2] = n3;
          for (int c = 0; c < 3; ++c) g[n].G[c] = G[c];
          g[n].G2 = G2;
          ++n;
        }
      }
  qsort(g, n, sizeof(orc_gvec), cmp_gvec);
  *ng = n;
  return g;
}

/* Index of -G for every G (the set is symmetric). */
static int *minus_index(const orc_gvec *g, int ng) {
  int *mi = (int *)malloc(sizeof(int) * ng);
  for (int i = 0; i < ng; ++i) {
    orc_gvec key;
    for (int c = 0; c < 3; ++c) key.n[c] = -g[i].n[c];
    const orc_gvec *hit = (const orc_gvec *)bsearch(&key, g, ng, sizeof(orc_gvec), cmp_gvec);
    mi[i] = hit ? (int)(hit - g) : -1;
  }
  return mi;
}

/* Primitive pairs (a in cell 0, b in cell L) with K >= eps_pair (and |A-B-L| <= r_max). */
static orc_pair *make_pairs(const orc_sys *s, int *np) {
  size_t cap = 1024, n = 0;
  orc_pair *pl = (orc_pair *)malloc(sizeof(orc_pair) * cap);
  double lneps = -log(s->eps_pair);
  for (int sa = 0; sa < s->nshell; ++sa)
    for (int sb = 0; sb < s->nshell; ++sb) {
      const double *RA = s->xyz + 3 * s->sh_atom[sa];
      const double *RB = s->xyz + 3 * s->sh_atom[sb];
      double d[3] = {RA[0] - RB[0], RA[1] - RB[1], RA[2] - RB[2]};
      for (int ia = s->pr_off[sa]; ia < s->pr_off[sa + 1]; ++ia)
        for (int ib = s->pr_off[sb]; ib < s->pr_off[sb + 1]; ++ib) {
          double aa = s->exps[ia], ab = s->exps[ib];
          double mu = aa * ab / (aa + ab);
          double R = sqrt(lneps / mu);
          if (s->r_max > 0 && s->r_max < R) R = s->r_max;
          int lo[3], hi[3];
          for (int i = 0; i < 3; ++i) {
            /* m_i = b_i . L / 2pi and |b_i . (L - d)| <= |b_i| R */
            double bd = s->B[0][i] * d[0] + s->B[1][i] * d[1] + s->B[2][i] * d[2];
            double bn = sqrt(s->B[0][i] * s->B[0][i] + s->B[1][i] * s->B[1][i] + s->B[2][i] * s->B[2][i]);
            lo[i] = (int)floor((bd - bn * R) / (2.0 * ORC_PI)) - 1;
            hi[i] = (int)ceil((bd + bn * R) / (2.0 * ORC_PI)) + 1;
          }
          for (int m1 = lo[0]; m1 <= hi[0]; ++m1)
            for (int m2 = lo[1]; m2 <= hi[1]; ++m2)
              for (int m3 = lo[2]; m3 <= hi[2]; ++m3) {
                double L[3], r2 = 0.0;
                for (int c = 0; c < 3; ++c) {
                  L[c] = s->A[c][0] * m1 + s->A[c][1] * m2 + s->A[c][2] * m3;
                  double x = d[c] - L[c];
                  r2 += x * x;
                }
                double K = exp(-mu * r2);
                if (!(K >= s->eps_pair)) continue;
                if (s->r_max > 0 && sqrt(r2) > s->r_max) continue;
                if (n == cap) {
                  cap *= 2;
                  pl = (orc_pair *)realloc(pl, sizeof(orc_pair) * cap);
                }
                orc_pair *q = &pl[n++];
                q->sa = sa;
                q->sb = sb;
                q->ia = ia;
                q->ib = ib;
                q->m[0] = m1;
                q->m[1] = m2;
                q->m[2] = m3;
                for (int c = 0; c < 3; ++c) q->L[c] = L[c];
              }
        }
    }
  *np = (int)n;
  return pl;
}

/* e^{i k.L} for mesh point kidx and image m: k.L = 2 pi sum_i m^k_i m_i / n_i. */
static zd kphase(const orc_sys *s, int kidx, const int m[3]) {
  int km[3];
  km[2] = kidx % s->kmesh[2];
  km[1] = (kidx / s->kmesh[2]) % s->kmesh[1];
  km[0] = kidx / (s->kmesh[2] * s->kmesh[1]);
  double t = 0.0;
  for (int i = 0; i < 3; ++i) t += (double)km[i] * m[i] / s->kmesh[i];
  double a = 2.0 * ORC_PI * t;
  return cos(a) + I * sin(a);
}

/* F block of a primitive pair at one G: Fab[i*ncb + j] for components i of a, j of b.
 * B' = centre of b (already shifted by L).  Includes c_a c_b N_a N_b.
 * dA/dB (optional): derivatives with respect to the centres, [3][nca*ncb]. */
static void pair_ft_block(int la, int lb, double aa, const double *RA, double ab, const double *RB,
                          double pref, const double *G, zd *F, zd *dA, zd *dB) {
  int deriv = (dA != NULL);
  int imax = la + deriv, jmax = lb + deriv;
  zd f[3][ORC_LMAX + 1][ORC_LMAX + 1];
  for (int x = 0; x < 3; ++x) ft_axis(imax, jmax, aa, RA[x], ab, RB[x], G[x], f[x]);
  int ca[21][3], cb[21][3];
  cart_list(la, ca);
  cart_list(lb, cb);
  int nca = ncart_of(la), ncb = ncart_of(lb);
  for (int i = 0; i < nca; ++i)
    for (int j = 0; j < ncb; ++j) {
      int *a = ca[i], *b = cb[j];
      F[i * ncb + j] = pref * f[0][a[0]][b[0]] * f[1][a[1]][b[1]] * f[2][a[2]][b[2]];
      if (!deriv) continue;
      for (int x = 0; x < 3; ++x) {
        int y = (x + 1) % 3, z = (x + 2) % 3;
        zd other = f[y][a[y]][b[y]] * f[z][a[z]][b[z]];
        /* d/dA_x (x-A_x)^l e^{-a (x-A_x)^2} = 2a (x-A_x)^{l+1}(...) - l (x-A_x)^{l-1}(...) */
        zd da = 2.0 * aa * f[x][a[x] + 1][b[x]];
        if (a[x] > 0) da -= (double)a[x] * f[x][a[x] - 1][b[x]];
        zd db = 2.0 * ab * f[x][a[x]][b[x] + 1];
        if (b[x] > 0) db -= (double)b[x] * f[x][a[x]][b[x] - 1];
        dA[x * nca * ncb + i * ncb + j] = pref * da * other;
        dB[x * nca * ncb + i * ncb + j] = pref * db * other;
      }
    }
}

/* ------------------------------------------------------------------------- */
/* per-pair reciprocal-space cut (section "Integral screening")               */
/* ------------------------------------------------------------------------- */

/* Screening objective of a primitive pair at |G| = G (eq. "AFT screening obj"
 * with eq. "eta_munu"):
 *   eps(G) = 8 pi eta G (4 pi / G^2) e^{-G^2/4w^2} |F|_inf(G),
 *   eta = [1/(a_a + a_b) + 1/w^2]^{-1},
 * |F|_inf(G): the largest modulus of the pair transform over the Cartesian
 * components of the shell pair and over G along x, y and z (the paper names the
 * infinity norm of the exact transform without fixing the directions). */
static double screen_objective(int la, int lb, double aa, const double *RA, double ab, const double *RB,
                               double pref, double omega, double G) {
  zd F[441];
  double fmax = 0.0;
  int n = ncart_of(la) * ncart_of(lb);
  for (int d = 0; d < 3; ++d) {
    double Gv[3] = {0.0, 0.0, 0.0};
    Gv[d] = G;
    pair_ft_block(la, lb, aa, RA, ab, RB, pref, Gv, F, NULL, NULL);
    for (int e = 0; e < n; ++e)
      if (cabs(F[e]) > fmax) fmax = cabs(F[e]);
  }
  double eta = 1.0 / (1.0 / (aa + ab) + 1.0 / (omega * omega));
  return 8.0 * ORC_PI * eta * G * (4.0 * ORC_PI / (G * G)) * exp(-G * G / (4.0 * omega * omega)) * fmax;
}

/* Cut radius of one pair: the objective falls below eps_G for good from here up
 * to the global cutoff.  From the global cutoff downwards in 256 equal steps to
 * the first G where the objective is >= eps_G (G -> 0 always is: the objective
 * grows like 1/G), then 60 bisection steps on that step; the cut is the
 * bracket's upper end.  The global cutoff itself if the objective is >= eps_G
 * there. */
static double pair_cut(int la, int lb, double aa, const double *RA, double ab, const double *RB, double pref,
                       double omega, double eps_G) {
  double gglob = 2.0 * omega * sqrt(-log(eps_G));
  if (screen_objective(la, lb, aa, RA, ab, RB, pref, omega, gglob) >= eps_G) return gglob;
  double hi = gglob, lo = 0.0;
  for (int k = 1; k < 256; ++k) {
    double G = gglob * (1.0 - k / 256.0);
    if (screen_objective(la, lb, aa, RA, ab, RB, pref, omega, G) >= eps_G) {
      lo = G;
      break;
    }
    hi = G;
  }
  for (int it = 0; it < 60; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid > 0.0 && screen_objective(la, lb, aa, RA, ab, RB, pref, omega, mid) >= eps_G)
      lo = mid;
    else
      hi = mid;
  }
  return hi;
}

static int cmp_block(const orc_pair *x, const orc_pair *y) {
  if (x->sa != y->sa) return x->sa < y->sa ? -1 : 1;
  if (x->sb != y->sb) return x->sb < y->sb ? -1 : 1;
  for (int i = 0; i < 3; ++i)
    if (x->m[i] != y->m[i]) return x->m[i] < y->m[i] ? -1 : 1;
  return 0;
}

static const orc_pair *g_sort_pairs;
static int cmp_pair_index(const void *a, const void *b) {
  int i = *(const int *)a, j = *(const int *)b;
  int c = cmp_block(&g_sort_pairs[i], &g_sort_pairs[j]);
  return c ? c : (i < j ? -1 : i > j);
}

/* Squared cut radius of every pair: each block (shell a, shell b, image m) takes
 * the cut of its most compact primitive pair (largest a_a + a_b; the first of
 * equal ones), which the paper uses for a whole contracted shell pair. */
static double *pair_cuts2(const orc_sys *s, const orc_pair *pl, int np) {
  double *gc2 = (double *)malloc(sizeof(double) * (np > 0 ? np : 1));
  int *idx = (int *)malloc(sizeof(int) * (np > 0 ? np : 1));
  for (int q = 0; q < np; ++q) idx[q] = q;
  g_sort_pairs = pl;
  qsort(idx, np, sizeof(int), cmp_pair_index);
  for (int g0 = 0; g0 < np;) {
    int g1 = g0 + 1;
    while (g1 < np && cmp_block(&pl[idx[g0]], &pl[idx[g1]]) == 0) ++g1;
    int best = idx[g0];
    for (int k = g0 + 1; k < g1; ++k) {
      const orc_pair *P = &pl[idx[k]];
      if (s->exps[P->ia] + s->exps[P->ib] > s->exps[pl[best].ia] + s->exps[pl[best].ib]) best = idx[k];
    }
    const orc_pair *P = &pl[best];
    int la = s->sh_l[P->sa], lb = s->sh_l[P->sb];
    const double *RA = s->xyz + 3 * s->sh_atom[P->sa];
    const double *RB0 = s->xyz + 3 * s->sh_atom[P->sb];
    double RB[3] = {RB0[0] + P->L[0], RB0[1] + P->L[1], RB0[2] + P->L[2]};
    double pref = fabs(s->coefs[P->ia] * s->coefs[P->ib]) * norm_of(la, s->exps[P->ia]) * norm_of(lb, s->exps[P->ib]);
    double c = pair_cut(la, lb, s->exps[P->ia], RA, s->exps[P->ib], RB, pref, s->omega, s->eps_G);
    for (int k = g0; k < g1; ++k) gc2[idx[k]] = c * c;
    g0 = g1;
  }
  free(idx);
  return gc2;
}

/* ------------------------------------------------------------------------- */
/* exported entry points                                                      */
/* ------------------------------------------------------------------------- */

/* Screening objective and cut radius of one primitive pair (unit contraction
 * coefficients) for pins: out[0] = eps(G), out[1] = cut radius. */
void orc_pair_cut(int la, int lb, double aa, const double *RA, double ab, const double *RB, double omega,
                  double eps_G, double G, double *out) {
  double pref = norm_of(la, aa) * norm_of(lb, ab);
  out[0] = G > 0.0 ? screen_objective(la, lb, aa, RA, ab, RB, pref, omega, G) : HUGE_VAL;
  out[1] = pair_cut(la, lb, aa, RA, ab, RB, pref, omega, eps_G);
}

/* Sizes of the lists the oracle builds (diagnostics). */
int orc_sizes(const double *lattice, int natm, const double *xyz, int nshell, const int *shell_atom,
              const int *shell_l, const int *shell_nprim, const double *exps, const double *coefs,
              const int *kmesh, double omega, double eps_pair, double eps_G, double r_max,
              int64_t *out /* [4]: nG, npairs, nbf, nk */) {
  orc_sys s;
  if (sys_setup(&s, lattice, natm, xyz, nshell, shell_atom, shell_l, shell_nprim, exps, coefs,
                kmesh, omega, eps_pair, eps_G, r_max))
    return -1;
  int ng, np;
  orc_gvec *g = make_gvecs(&s, &ng);
  orc_pair *pl = make_pairs(&s, &np);
  out[0] = ng;
  out[1] = np;
  out[2] = s.nbf;
  out[3] = s.nk;
  free(g);
  free(pl);
  sys_free(&s);
  return 0;
}

/* The screened pair list itself (diagnostics): out[q] = (sa, sb, ia, ib, m1, m2, m3)
 * for q < min(count, maxp), in the order the oracle sums them.  Lets a
 * finite-difference test confirm that a displaced geometry keeps the same list
 * (the gradient is defined at a fixed pair list).  Returns the pair count, or
 * -1 on bad input. */
int orc_pairs(const double *lattice, int natm, const double *xyz, int nshell, const int *shell_atom,
              const int *shell_l, const int *shell_nprim, const double *exps, const double *coefs,
              const int *kmesh, double omega, double eps_pair, double eps_G, double r_max,
              int *out, int maxp) {
  orc_sys s;
  if (sys_setup(&s, lattice, natm, xyz, nshell, shell_atom, shell_l, shell_nprim, exps, coefs,
                kmesh, omega, eps_pair, eps_G, r_max))
    return -1;
  int np;
  orc_pair *pl = make_pairs(&s, &np);
  for (int q = 0; q < np && q < maxp; ++q) {
    int *o = out + 7 * (size_t)q;
    o[0] = pl[q].sa;
    o[1] = pl[q].sb;
    o[2] = pl[q].ia;
    o[3] = pl[q].ib;
    for (int c = 0; c < 3; ++c) o[4 + c] = pl[q].m[c];
  }
  free(pl);
  sys_free(&s);
  return np;
}

/* Un-normalised 1D pair transform f[i][j] at G (for quadrature pins). */
void orc_ft_axis(int i, int j, double aa, double Ax, double ab, double Bx, double G, double *out) {
  zd f[ORC_LMAX + 1][ORC_LMAX + 1];
  ft_axis(i, j, aa, Ax, ab, Bx, G, f);
  out[0] = creal(f[i][j]);
  out[1] = cimag(f[i][j]);
}

/* Normalised pair transform block (unit contraction coefficients) at one G,
 * complex interleaved [ncart(la)][ncart(lb)]; optional centre derivatives
 * dA, dB: [3][ncart(la)][ncart(lb)] complex. */
void orc_pair_ft(int la, int lb, double aa, const double *RA, double ab, const double *RB,
                 const double *G, double *out, double *dA, double *dB) {
  double pref = norm_of(la, aa) * norm_of(lb, ab);
  int n = ncart_of(la) * ncart_of(lb);
  zd *F = (zd *)malloc(sizeof(zd) * n * 7);
  zd *gA = dA ? F + n : NULL, *gB = dA ? F + 4 * n : NULL;
  pair_ft_block(la, lb, aa, RA, ab, RB, pref, G, F, gA, gB);
  memcpy(out, F, sizeof(zd) * n);
  if (dA) {
    memcpy(dA, gA, sizeof(zd) * 3 * n);
    memcpy(dB, gB, sizeof(zd) * 3 * n);
  }
  free(F);
}

/*
 * Long-range J for one density.
 *   Dk      complex128 interleaved [nk][nbf][nbf]
 *   Jk      out, same layout (NULL: skip J(k) and E3)
 *   energy  out [6]: E(real space), E(G space), E(k space),
 *           max|Im J(L)|, max|J(L)|, Omega*rho(0)  (rho(0) from F at G = 0)
 *   rho     out [maxG][2] and miller [maxG][3] (NULL: skip); nG_out gets |G set|
 *   grad    out [natm][3] (NULL: skip)
 *   pair_gcut  1: per-pair G cuts;  alpha_cut  > 0: compact/diffuse classification
 *   (rho out is then rho_C + rho_D)
 * Returns 0, or -1 on bad input, -2 when maxG is too small.
 */
int orc_build_j(const double *lattice, int natm, const double *xyz, int nshell,
                const int *shell_atom, const int *shell_l, const int *shell_nprim,
                const double *exps, const double *coefs, const int *kmesh, double omega,
                double eps_pair, double eps_G, double r_max, const double *Dk_, double *Jk_,
                double *energy, double *rho_out, int *miller, int maxG, int *nG_out,
                double *grad, int nthreads, int pair_gcut, double alpha_cut) {
  orc_sys s;
  if (sys_setup(&s, lattice, natm, xyz, nshell, shell_atom, shell_l, shell_nprim, exps, coefs,
                kmesh, omega, eps_pair, eps_G, r_max))
    return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  const zd *Dk = (const zd *)Dk_;
  zd *Jk = (zd *)Jk_;
  int nbf = s.nbf, nk = s.nk;
  int ng, np;
  orc_gvec *g = make_gvecs(&s, &ng);
  int *mi = minus_index(g, ng);
  orc_pair *pl = make_pairs(&s, &np);
  if (nG_out) *nG_out = ng;
  if (rho_out && ng > maxG) {
    free(g);
    free(mi);
    free(pl);
    sys_free(&s);
    return -2;
  }

  /* per-pair cut (section "Integral screening"): pair q sees only the G of the
   * set with |G|^2 <= gc2[q]; without it every pair sees the whole set */
  double *gc2 = pair_gcut ? pair_cuts2(&s, pl, np) : NULL;

  /* compact/diffuse classification: dd[q] = 1 for a pair of two diffuse
   * primitives (exponents below alpha_cut); DD pairs see the whole G set */
  char *dd = (char *)calloc(np > 0 ? np : 1, 1);
  for (int q = 0; q < np; ++q) {
    dd[q] = alpha_cut > 0.0 && exps[pl[q].ia] < alpha_cut && exps[pl[q].ib] < alpha_cut;
    if (gc2 && dd[q]) gc2[q] = HUGE_VAL;
  }

  /* per-pair block offsets, D(L) blocks and prefactors */
  int64_t *boff = (int64_t *)malloc(sizeof(int64_t) * (np + 1));
  boff[0] = 0;
  for (int q = 0; q < np; ++q)
    boff[q + 1] = boff[q] + (int64_t)ncart_of(shell_l[pl[q].sa]) * ncart_of(shell_l[pl[q].sb]);
  zd *DL = (zd *)malloc(sizeof(zd) * boff[np]);
  double *JL = (double *)calloc(boff[np], sizeof(double));
  double *pref = (double *)malloc(sizeof(double) * np);
  double wk = 1.0 / nk;
#pragma omp parallel for schedule(dynamic, 64)
  for (int q = 0; q < np; ++q) {
    const orc_pair *P = &pl[q];
    int la = shell_l[P->sa], lb = shell_l[P->sb];
    int nca = ncart_of(la), ncb = ncart_of(lb);
    pref[q] = coefs[P->ia] * coefs[P->ib] * norm_of(la, exps[P->ia]) * norm_of(lb, exps[P->ib]);
    for (int i = 0; i < nca; ++i)
      for (int j = 0; j < ncb; ++j) {
        int mu = s.sh_off[P->sa] + i, nu = s.sh_off[P->sb] + j;
        zd acc = 0.0;
        for (int k = 0; k < nk; ++k) acc += wk * kphase(&s, k, P->m) * Dk[(int64_t)k * nbf * nbf + (int64_t)mu * nbf + nu];
        DL[boff[q] + i * ncb + j] = acc;
      }
  }

  /* rho(G) = (1/Omega) sum_pairs D_ab(L) F_abL(G), split by pair class:
   * rho holds the compact pairs' part, rhoD the DD pairs' part */
  zd *rho = (zd *)malloc(sizeof(zd) * ng);
  zd *rhoD = (zd *)malloc(sizeof(zd) * ng);
#pragma omp parallel for schedule(dynamic, 1)
  for (int ig = 0; ig < ng; ++ig) {
    zd F[441];
    zd acc = 0.0, accD = 0.0;
    for (int q = 0; q < np; ++q) {
      const orc_pair *P = &pl[q];
      int la = shell_l[P->sa], lb = shell_l[P->sb];
      const double *RA = xyz + 3 * shell_atom[P->sa];
      const double *RB0 = xyz + 3 * shell_atom[P->sb];
      double RB[3] = {RB0[0] + P->L[0], RB0[1] + P->L[1], RB0[2] + P->L[2]};
      if (gc2 && g[ig].G2 > gc2[q]) continue;
      pair_ft_block(la, lb, exps[P->ia], RA, exps[P->ib], RB, pref[q], g[ig].G, F, NULL, NULL);
      int n = ncart_of(la) * ncart_of(lb);
      zd *a = dd[q] ? &accD : &acc;
      for (int e = 0; e < n; ++e) *a += DL[boff[q] + e] * F[e];
    }
    rho[ig] = acc / s.omega_vol;
    rhoD[ig] = accD / s.omega_vol;
  }

  /* v(G) (long range), vf(G) (full range) and the G-space energy */
  double *v = (double *)malloc(sizeof(double) * ng);
  double *vf = (double *)malloc(sizeof(double) * ng);
  double e_g = 0.0;
  for (int ig = 0; ig < ng; ++ig) {
    v[ig] = 4.0 * ORC_PI * exp(-g[ig].G2 / (4.0 * omega * omega)) / g[ig].G2;
    vf[ig] = 4.0 * ORC_PI / g[ig].G2;
    e_g += v[ig] * creal(rho[ig] * rho[mi[ig]]);
    /* interactions with a DD side, in full */
    e_g += vf[ig] * creal(rho[ig] * rhoD[mi[ig]] + rhoD[ig] * rho[mi[ig]] + rhoD[ig] * rhoD[mi[ig]]);
  }
  e_g *= 0.5 * s.omega_vol;

  /* J_ab(L) = sum_G v(G) rho(-G) F_abL(G) */
  double max_im = 0.0, max_j = 0.0, e_r = 0.0;
  double *gth = NULL;
  int nth = 1;
#ifdef _OPENMP
  nth = omp_get_max_threads();
#endif
  if (grad) gth = (double *)calloc((size_t)nth * natm * 3, sizeof(double));
#pragma omp parallel reduction(max : max_im, max_j) reduction(+ : e_r)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    zd F[441], dA[3 * 441], dB[3 * 441], Jc[441];
#pragma omp for schedule(dynamic, 16)
    for (int q = 0; q < np; ++q) {
      const orc_pair *P = &pl[q];
      int la = shell_l[P->sa], lb = shell_l[P->sb];
      int n = ncart_of(la) * ncart_of(lb);
      const double *RA = xyz + 3 * shell_atom[P->sa];
      const double *RB0 = xyz + 3 * shell_atom[P->sb];
      double RB[3] = {RB0[0] + P->L[0], RB0[1] + P->L[1], RB0[2] + P->L[2]};
      for (int e = 0; e < n; ++e) Jc[e] = 0.0;
      double gA[3] = {0, 0, 0}, gB[3] = {0, 0, 0};
      for (int ig = 0; ig < ng; ++ig) {
        if (gc2 && g[ig].G2 > gc2[q]) continue;
        /* V(-G) of the pair's class: V_C for compact pairs, V_D for DD pairs */
        zd w = dd[q] ? vf[ig] * (rho[mi[ig]] + rhoD[mi[ig]]) : v[ig] * rho[mi[ig]] + vf[ig] * rhoD[mi[ig]];
        pair_ft_block(la, lb, exps[P->ia], RA, exps[P->ib], RB, pref[q], g[ig].G, F,
                      grad ? dA : NULL, grad ? dB : NULL);
        for (int e = 0; e < n; ++e) Jc[e] += w * F[e];
        if (grad) {
          for (int x = 0; x < 3; ++x) {
            zd sa_ = 0.0, sb_ = 0.0;
            for (int e = 0; e < n; ++e) {
              sa_ += DL[boff[q] + e] * dA[x * n + e];
              sb_ += DL[boff[q] + e] * dB[x * n + e];
            }
            gA[x] += creal(w * sa_);
            gB[x] += creal(w * sb_);
          }
        }
      }
      for (int e = 0; e < n; ++e) {
        if (fabs(cimag(Jc[e])) > max_im) max_im = fabs(cimag(Jc[e]));
        if (fabs(creal(Jc[e])) > max_j) max_j = fabs(creal(Jc[e]));
        JL[boff[q] + e] = creal(Jc[e]);
        e_r += 0.5 * creal(DL[boff[q] + e]) * creal(Jc[e]) - 0.5 * cimag(DL[boff[q] + e]) * cimag(Jc[e]);
      }
      if (grad) {
        int A_ = shell_atom[P->sa], B_ = shell_atom[P->sb];
        for (int x = 0; x < 3; ++x) {
          gth[((size_t)tid * natm + A_) * 3 + x] += gA[x];
          gth[((size_t)tid * natm + B_) * 3 + x] += gB[x];
        }
      }
    }
  }
  if (grad) {
    for (int a = 0; a < natm * 3; ++a) {
      double t = 0.0;
      for (int th = 0; th < nth; ++th) t += gth[(size_t)th * natm * 3 + a];
      grad[a] = t;
    }
    free(gth);
  }

  /* J(k) = sum_L e^{ik.L} J(L) and the k-space energy */
  double e_k = 0.0;
  if (Jk) {
    memset(Jk, 0, sizeof(zd) * (size_t)nk * nbf * nbf);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nk; ++k) {
      zd *Jkk = Jk + (int64_t)k * nbf * nbf;
      for (int q = 0; q < np; ++q) {
        const orc_pair *P = &pl[q];
        int ncb = ncart_of(shell_l[P->sb]), nca = ncart_of(shell_l[P->sa]);
        zd ph = kphase(&s, k, P->m);
        for (int i = 0; i < nca; ++i)
          for (int j = 0; j < ncb; ++j) {
            int mu = s.sh_off[P->sa] + i, nu = s.sh_off[P->sb] + j;
            Jkk[(int64_t)mu * nbf + nu] += ph * JL[boff[q] + i * ncb + j];
          }
      }
    }
    for (int k = 0; k < nk; ++k)
      for (int64_t e = 0; e < (int64_t)nbf * nbf; ++e)
        e_k += creal(Dk[(int64_t)k * nbf * nbf + e] * Jk[(int64_t)k * nbf * nbf + e]);
    e_k *= 0.5 * wk;
  }

  /* Omega * rho(0) from the transform at G = 0 (0 is not in the G set) */
  double q0 = 0.0;
  {
    zd F[441];
    double G0[3] = {0, 0, 0};
    for (int q = 0; q < np; ++q) {
      const orc_pair *P = &pl[q];
      int la = shell_l[P->sa], lb = shell_l[P->sb];
      const double *RA = xyz + 3 * shell_atom[P->sa];
      const double *RB0 = xyz + 3 * shell_atom[P->sb];
      double RB[3] = {RB0[0] + P->L[0], RB0[1] + P->L[1], RB0[2] + P->L[2]};
      pair_ft_block(la, lb, exps[P->ia], RA, exps[P->ib], RB, pref[q], G0, F, NULL, NULL);
      int n = ncart_of(la) * ncart_of(lb);
      for (int e = 0; e < n; ++e) q0 += creal(DL[boff[q] + e] * F[e]);
    }
  }

  if (energy) {
    energy[0] = e_r;
    energy[1] = e_g;
    energy[2] = e_k;
    energy[3] = max_im;
    energy[4] = max_j;
    energy[5] = q0;
  }
  if (rho_out) {
    for (int ig = 0; ig < ng; ++ig) {
      rho_out[2 * ig] = creal(rho[ig] + rhoD[ig]);
      rho_out[2 * ig + 1] = cimag(rho[ig] + rhoD[ig]);
      if (miller)
        for (int c = 0; c < 3; ++c) miller[3 * ig + c] = g[ig].n[c];
    }
  }
  free(gc2);
  free(dd);
  free(rho);
  free(rhoD);
  free(v);
  free(vf);
  free(DL);
  free(JL);
  free(pref);
  free(boff);
  free(g);
  free(mi);
  free(pl);
  sys_free(&s);
  return 0;
}
