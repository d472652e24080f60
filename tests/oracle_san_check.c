/* The FP64 oracle (oracle/pwdf_oracle.c) run as a plain program, for a build
 * with the address and undefined-behaviour sanitizers.  Reads the problem as
 * whitespace-separated text (lattice (9), natm and xyz, nshell and shell atoms,
 * shell l, shell primitive counts, primitive count and exponents, coefficients,
 * kmesh (3), omega, eps_pair, eps_G, r_max, pair_gcut, alpha_cut) and D(k) as raw
 * complex128 [nk][nbf][nbf] from a second file; computes J(k), rho(G), E_J and
 * the gradient in one call (single thread) and prints
 * "E_G <e> E_R <e> sumJ <s> sumrho <s> sumgrad <s>".  Exit status non-zero on a
 * read or oracle error. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_sizes(const double *lattice, int natm, const double *xyz, int nshell, const int *shell_atom,
              const int *shell_l, const int *shell_nprim, const double *exps, const double *coefs,
              const int *kmesh, double omega, double eps_pair, double eps_G, double r_max, int64_t *out);
int orc_build_j(const double *lattice, int natm, const double *xyz, int nshell, const int *shell_atom,
                const int *shell_l, const int *shell_nprim, const double *exps, const double *coefs,
                const int *kmesh, double omega, double eps_pair, double eps_G, double r_max, const double *Dk,
                double *Jk, double *energy, double *rho_out, int *miller, int maxG, int *nG_out, double *grad,
                int nthreads, int pair_gcut, double alpha_cut);

static int read_ints(FILE *f, int *v, int n) {
  for (int i = 0; i < n; ++i)
    if (fscanf(f, "%d", &v[i]) != 1) return 1;
  return 0;
}

static int read_dbls(FILE *f, double *v, int n) {
  for (int i = 0; i < n; ++i)
    if (fscanf(f, "%lf", &v[i]) != 1) return 1;
  return 0;
}

int main(int argc, char **argv) {
  if (argc < 3) return 2;
  FILE *f = fopen(argv[1], "r");
  if (!f) return 2;
  double lat[9], omega, eps_pair, eps_G, r_max, alpha_cut;
  int natm, nshell, nprim, kmesh[3], gcut;
  if (read_dbls(f, lat, 9) || fscanf(f, "%d", &natm) != 1) return 2;
  double *xyz = malloc(sizeof(double) * 3 * natm);
  if (read_dbls(f, xyz, 3 * natm) || fscanf(f, "%d", &nshell) != 1) return 2;
  int *sa = malloc(sizeof(int) * nshell), *sl = malloc(sizeof(int) * nshell), *sn = malloc(sizeof(int) * nshell);
  if (read_ints(f, sa, nshell) || read_ints(f, sl, nshell) || read_ints(f, sn, nshell)) return 2;
  if (fscanf(f, "%d", &nprim) != 1) return 2;
  double *ex = malloc(sizeof(double) * nprim), *co = malloc(sizeof(double) * nprim);
  if (read_dbls(f, ex, nprim) || read_dbls(f, co, nprim) || read_ints(f, kmesh, 3)) return 2;
  if (fscanf(f, "%lf %lf %lf %lf %d %lf", &omega, &eps_pair, &eps_G, &r_max, &gcut, &alpha_cut) != 6) return 2;
  fclose(f);
  int64_t sz[4];
  if (orc_sizes(lat, natm, xyz, nshell, sa, sl, sn, ex, co, kmesh, omega, eps_pair, eps_G, r_max, sz)) return 3;
  const int64_t nG = sz[0], nbf = sz[2], nk = sz[3], n = 2 * nk * nbf * nbf;
  double *D = malloc(sizeof(double) * n), *J = malloc(sizeof(double) * n);
  double *rho = malloc(sizeof(double) * 2 * (nG > 0 ? nG : 1)), *grad = malloc(sizeof(double) * 3 * natm);
  int *mil = malloc(sizeof(int) * 3 * (nG > 0 ? nG : 1));
  FILE *fd = fopen(argv[2], "rb");
  if (!fd || fread(D, sizeof(double), (size_t)n, fd) != (size_t)n) return 2;
  fclose(fd);
  double e[6];
  int nG_out = 0;
  if (orc_build_j(lat, natm, xyz, nshell, sa, sl, sn, ex, co, kmesh, omega, eps_pair, eps_G, r_max, D, J, e, rho,
                  mil, (int)nG, &nG_out, grad, 1, gcut, alpha_cut))
    return 3;
  double sj = 0.0, sr = 0.0, sg = 0.0;
  for (int64_t i = 0; i < n; ++i) sj += J[i] * J[i];
  for (int64_t i = 0; i < 2 * (int64_t)nG_out; ++i) sr += rho[i] * rho[i];
  for (int i = 0; i < 3 * natm; ++i) sg += grad[i] * grad[i];
  printf("E_G %.17g E_R %.17g sumJ %.17g sumrho %.17g sumgrad %.17g\n", e[1], e[0], sj, sr, sg);
  free(xyz), free(sa), free(sl), free(sn), free(ex), free(co), free(D), free(J), free(rho), free(grad), free(mil);
  return 0;
}
