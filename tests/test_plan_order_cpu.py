"""The pair order of the rho pass (plan.cpp), checked on the host: the low
classes (L <= 2) are walked in order of p so that a wave can keep the
p-dependent start factors of its previous pair; the density transform writes
each pair's coefficients at its rank in that walk.  The checker builds the plan
from the library's own plan.cpp (compiled for the host) and verifies that the
rank is a permutation within every class, that the reordered pair records equal
the stored ones, that the sort is by p and stable, and that the high classes keep
storage order.  Cells: the cubic two-atom cell (s, p, d shells) and the rock-salt
slab (up to f shells, classes up to (3,3))."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2509_16460_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2509_16460_amd", "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("plan") / "plan_order_check")
    subprocess.check_call([gxx, "-O2", "-std=c++17", "-D__host__=", "-D__device__=", "-D__forceinline__=inline",
                           "-I", CSRC, "-I", INCLUDE, os.path.join(HERE, "plan_order_check.cpp"),
                           os.path.join(CSRC, "plan.cpp"), "-o", exe])
    return exe


def write_problem(p, path):
    vals = [*np.asarray(p.lattice).ravel(), p.natm, *np.asarray(p.xyz).ravel(), p.nshell, *p.shell_atom,
            *p.shell_l, *p.shell_nprim, len(p.exps), *p.exps, *p.coefs, *p.kmesh, p.omega, p.eps_pair, p.eps_G,
            p.r_max]
    with open(path, "w") as f:
        f.write(" ".join(repr(float(v)) if isinstance(v, (float, np.floating)) else str(int(v)) for v in vals))


@pytest.mark.parametrize("cfg", [1, 4])
def test_rho_walk_order(checker, tmp_path, cfg):
    p = synth.config_problem(cfg)
    path = str(tmp_path / "problem.txt")
    write_problem(p, path)
    out = subprocess.run([checker, path], capture_output=True, text=True)
    print(out.stdout.strip())
    assert out.returncode == 0, out.stdout + out.stderr
    words = out.stdout.split()
    assert int(words[1]) > 0 and words[-1] == "0"
