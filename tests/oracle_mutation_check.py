#!/usr/bin/env python
"""Mutation check of the oracle pins (CPU only; not collected by pytest).

Each entry plants one plausible mistake in a copy of oracle/pwdf_oracle.c (a
dropped factor, a wrong sign, a transposed index, a wrong constant), builds the
copy into a temporary directory and runs the CPU pin and invariant tests against
it (PWDF_ORACLE_LIB).  A mutant is "killed" when at least one of those tests
fails.  The committed oracle itself is never modified.

    python tests/oracle_mutation_check.py            # all mutants
    python tests/oracle_mutation_check.py herm xpb   # a subset
"""
import os
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pwdf_oracle.c")

# name: (exact text in the oracle, replacement, what the mistake is)
MUTANTS = {
    "binom": ("s += binom(i, ii) * binom(j, jj) * pow(XPA, i - ii)", "s += binom(i, ii) * pow(XPA, i - ii)",
              "dropped binomial factor of centre b in the Gaussian-product expansion"),
    "xpb": ("double XPA = P - Ax, XPB = P - Bx;", "double XPA = P - Ax, XPB = Bx - P;",
            "sign of P - B in the Gaussian-product expansion"),
    "herm": ("H[n] = 2.0 * x * H[n - 1] - 2.0 * (n - 1) * H[n - 2];", "H[n] = 2.0 * x * H[n - 1] - 2.0 * n * H[n - 2];",
             "wrong index in the Hermite recurrence"),
    "hstep": ("zd step = -I / (2.0 * sp);", "zd step = I / (2.0 * sp);",
              "the printed (+i) sign of the Cartesian-Gaussian transform"),
    "gpphase": ("zd ph = cos(G * P) - I * sin(G * P);", "zd ph = cos(G * P) + I * sin(G * P);",
                "sign of the e^{-iG.P} phase"),
    "norm": ("pow(4.0 * a, 0.5 * l) / sqrt(dfact(2 * l - 1))", "pow(2.0 * a, 0.5 * l) / sqrt(dfact(2 * l - 1))",
             "wrong Cartesian normalisation"),
    "dsum": ("double d[3] = {RA[0] - RB[0], RA[1] - RB[1], RA[2] - RB[2]};",
             "double d[3] = {RA[0] + RB[0], RA[1] - RB[1], RA[2] - RB[2]};", "sign of A - B in the pair screening"),
    "kphase": ("double a = 2.0 * ORC_PI * t;", "double a = -2.0 * ORC_PI * t;", "sign of e^{ik.L}"),
    "dtrans": ("Dk[(int64_t)k * nbf * nbf + (int64_t)mu * nbf + nu]", "Dk[(int64_t)k * nbf * nbf + (int64_t)nu * nbf + mu]",
               "transposed D(k) in D(L)"),
    "jkconj": ("        zd ph = kphase(&s, k, P->m);", "        zd ph = conj(kphase(&s, k, P->m));",
               "conjugated phase in J(k)"),
    "noomega": ("rho[ig] = acc / s.omega_vol;", "rho[ig] = acc;", "dropped 1/Omega in rho(G)"),
    "fourpi": ("v[ig] = 4.0 * ORC_PI * exp(", "v[ig] = 4.0 * exp(", "dropped pi in v(G)"),
    "omega": ("exp(-g[ig].G2 / (4.0 * omega * omega))", "exp(-g[ig].G2 / (2.0 * omega * omega))",
              "wrong range-separation exponent"),
    "ehalf": ("e_g *= 0.5 * s.omega_vol;", "e_g *= s.omega_vol;", "dropped 1/2 in the G-space energy"),
    "rhoplus": (": v[ig] * rho[mi[ig]] + vf[ig] * rhoD[mi[ig]];", ": v[ig] * rho[ig] + vf[ig] * rhoD[mi[ig]];",
                "V(G) instead of V(-G) in the J contraction"),
    "cdjv": ("zd w = dd[q] ? vf[ig] * (rho[mi[ig]] + rhoD[mi[ig]])", "zd w = dd[q] ? v[ig] * rho[mi[ig]] + vf[ig] * rhoD[mi[ig]]",
             "DD pairs contracted with the compact pairs' potential V_C"),
    "cdcross": ("e_g += vf[ig] * creal(rho[ig] * rhoD[mi[ig]] + rhoD[ig] * rho[mi[ig]]",
                "e_g += vf[ig] * creal(rho[ig] * rhoD[mi[ig]]",
                "one of the two compact-diffuse cross terms dropped from the G-space energy"),
    "cdvf": ("vf[ig] = 4.0 * ORC_PI / g[ig].G2;", "vf[ig] = v[ig];",
             "long-range kernel kept for the interactions with a DD side"),
    "cdle": ("exps[pl[q].ia] < alpha_cut && exps[pl[q].ib] < alpha_cut", "exps[pl[q].ia] < alpha_cut || exps[pl[q].ib] < alpha_cut",
             "CD pairs classified as diffuse"),
    "dgrad": ("if (a[x] > 0) da -= (double)a[x] * f[x][a[x] - 1][b[x]];",
              "if (a[x] > 0) da += (double)a[x] * f[x][a[x] - 1][b[x]];", "sign of the lowered term of the centre derivative"),
    "gswap": ("int A_ = shell_atom[P->sa], B_ = shell_atom[P->sb];",
              "int A_ = shell_atom[P->sb], B_ = shell_atom[P->sa];",
              "gradient of shell a assigned to the atom of shell b and vice versa"),
    "grhoplus": ("gA[x] += creal(w * sa_);\n            gB[x] += creal(w * sb_);",
                 "gA[x] += creal(v[ig] * rho[ig] * sa_);\n            gB[x] += creal(v[ig] * rho[ig] * sb_);",
                 "rho(G) instead of rho(-G) in the gradient only"),
    "gnod": ("sa_ += DL[boff[q] + e] * dA[x * n + e];", "sa_ += dA[x * n + e];",
             "dropped D weight of the shell-a centre derivative"),
    "gsignb": ("gB[x] += creal(w * sb_);", "gB[x] -= creal(w * sb_);",
               "sign of the shell-b centre derivative in the gradient"),
}

TESTS = ["tests/test_oracle_pins.py", "tests/test_oracle_invariants.py", "tests/test_oracle_grad.py",
         "tests/test_oracle_cd.py"]


def run(name, tmp):
    old, new, what = MUTANTS[name]
    src = open(SRC).read()
    if src.count(old) < 1:
        return name, "NOT APPLIED (text not found)", what
    path = os.path.join(tmp, f"{name}.c")
    with open(path, "w") as fh:
        fh.write(src.replace(old, new, 1))
    lib = os.path.join(tmp, f"{name}.so")
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off", "-std=c11", "-shared", "-fPIC",
                    "-o", lib, path, "-lm"], check=True)
    env = dict(os.environ, PWDF_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"] + TESTS, cwd=ROOT,
                       env=env, capture_output=True, text=True)
    last = (r.stdout.strip().splitlines() or ["?"])[-1]
    return name, ("killed: " + last) if r.returncode != 0 else ("SURVIVED: " + last), what


def main():
    names = sys.argv[1:] or list(MUTANTS)
    survived = 0
    with tempfile.TemporaryDirectory() as tmp:
        for n in names:
            name, res, what = run(n, tmp)
            survived += not res.startswith("killed")
            print(f"{name:8s} {res}  [{what}]", flush=True)
    sys.exit(1 if survived else 0)


if __name__ == "__main__":
    main()
