"""The pair order of the rho pass (plan.cpp), checked on the host: the low
classes (L <= 2) are walked in order of p so that a wave can keep the
p-dependent start factors of its previous pair; the density transform writes
each pair's coefficients at its rank in that walk.  The checker builds the plan
from the library's own plan.cpp (compiled for the host) and verifies that the
rank is a permutation within every class, that the reordered pair records equal
the stored ones, that the sort is by p and stable, and that the high classes keep
storage order.  Cells: the cubic two-atom cell (s, p, d shells) and the rock-salt
slab (up to f shells, classes up to (3,3)).

The same checker, built with the address and undefined-behaviour sanitizers
(g++ -fsanitize=address,undefined, no recovery), also runs the host planning code
over cells with per-pair cuts, DD pairs of the compact/diffuse classification
and the GPW grid lists, rebuilding the segments for every segment length the
tuner can pick and recounting the head of the G set for several weights."""
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


@pytest.fixture(scope="module")
def checker_san(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("plan_san") / "plan_order_check_san")
    subprocess.check_call([gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-static-libasan",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-D__host__=", "-D__device__=",
                           "-D__forceinline__=inline", "-I", CSRC, "-I", INCLUDE,
                           os.path.join(HERE, "plan_order_check.cpp"), os.path.join(CSRC, "plan.cpp"), "-o", exe])
    return exe


def write_problem(p, path):
    vals = [*np.asarray(p.lattice).ravel(), p.natm, *np.asarray(p.xyz).ravel(), p.nshell, *p.shell_atom,
            *p.shell_l, *p.shell_nprim, len(p.exps), *p.exps, *p.coefs, *p.kmesh, p.omega, p.eps_pair, p.eps_G,
            p.r_max, int(p.pair_gcut), float(p.alpha_cut), int(p.dd_gpw)]
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


SAN_CASES = {
    "cubic_cell": lambda: synth.config_problem(1),
    "slab_paircut": lambda: synth.config_problem(4).with_(pair_gcut=1),
    "diffuse_cd_paircut": lambda: synth.diffuse_problem().with_(pair_gcut=1),
    "diffuse_gpw": lambda: synth.diffuse_problem(a=11.0, natm=2).with_(dd_gpw=1),
}


@pytest.mark.parametrize("name", list(SAN_CASES))
def test_plan_under_sanitizers(checker_san, tmp_path, name):
    p = SAN_CASES[name]()
    path = str(tmp_path / "problem.txt")
    write_problem(p, path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([checker_san, path, "sweep"], capture_output=True, text=True, env=env, timeout=600)
    print(out.stdout.strip())
    assert out.returncode == 0, out.stdout + out.stderr[-4000:]
    assert "ERROR" not in out.stderr and "runtime error" not in out.stderr, out.stderr[-4000:]
    words = out.stdout.split()
    assert words[-1] == "0" and "sweep:" in words
    if p.alpha_cut > 0:
        assert int(words[words.index("dd") + 1]) > 0
    if p.dd_gpw:
        assert int(words[words.index("gpw") + 1]) > 0
