"""The FP64 oracle built with the address and undefined-behaviour sanitizers
(gcc -fsanitize=address,undefined, no recovery) and run as a plain program
(tests/oracle_san_check.c) on small cells: every class up to (3,3), per-pair cuts,
and the compact/diffuse classification.  Its E_J, J(k), rho(G) and gradient
must equal those of the ordinary build to rounding; the sanitizers must report
nothing."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_16460_amd import synth

from test_plan_order_cpu import write_problem

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle", "pwdf_oracle.c")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("oracle_san") / "oracle_san_check")
    subprocess.check_call([gcc, "-O1", "-g", "-std=c11", "-fno-fast-math", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-static-libasan", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", os.path.join(HERE, "oracle_san_check.c"), ORACLE, "-lm",
                           "-o", exe])
    return exe


def cd_sp_problem(a=5.0, seed=5):
    """Two atoms with s and p shells, one compact and one diffuse exponent each
    against alpha_cut = 0.125 (omega = 0.5): CC, CD and DD pairs."""
    rng = np.random.default_rng(seed)
    lat = np.array([[a, 0.0, 0.0], [0.3, 1.05 * a, 0.0], [-0.4, 0.5, 0.95 * a]])
    xyz = rng.uniform(0, 1, (2, 3)) @ lat
    ex = {0: [np.array([2.2, 0.11]), np.array([1.3, 0.115])]}
    prob = synth.build_problem("cd_sp", lat, xyz, [0, 0], ex, (1, 1, 1), 0.5, nelec=4.0, seed=seed)
    return prob.with_(alpha_cut=0.125)


CASES = {
    "spdf_k311": lambda: synth.small_problem(kind="spdf", seed=35, kmesh=(3, 1, 1), lmax=3, natm=2, lo=0.25, hi=40.0),
    "spd_k221_paircut": lambda: synth.small_problem(kind="spd", seed=33, kmesh=(2, 2, 1), lmax=2,
                                                    natm=2).with_(pair_gcut=1),
    "cd_sp": cd_sp_problem,
}


@pytest.mark.parametrize("name", list(CASES))
def test_oracle_under_sanitizers(checker, tmp_path, name):
    p = CASES[name]()
    D = synth.make_density(p, 140)
    ppath, dpath = str(tmp_path / "problem.txt"), str(tmp_path / "dk.bin")
    write_problem(p, ppath)
    np.ascontiguousarray(D, dtype=np.complex128).tofile(dpath)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([checker, ppath, dpath], capture_output=True, text=True, env=env, timeout=600)
    print(out.stdout.strip())
    assert out.returncode == 0, out.stdout + out.stderr[-4000:]
    assert "ERROR" not in out.stderr and "runtime error" not in out.stderr, out.stderr[-4000:]
    w = out.stdout.split()
    got = {w[i]: float(w[i + 1]) for i in range(0, len(w), 2)}
    ref = O.build_j(p, D, want_grad=True, nthreads=1)
    assert abs(got["E_G"] - ref["E_G"]) <= 1e-13 * max(1.0, abs(ref["E_G"]))
    assert abs(got["E_R"] - ref["E_real"]) <= 1e-13 * max(1.0, abs(ref["E_real"]))
    for key, val in (("sumJ", np.sum(np.abs(ref["J"]) ** 2)), ("sumrho", np.sum(np.abs(ref["rho"]) ** 2)),
                     ("sumgrad", np.sum(ref["grad"] ** 2))):
        assert abs(got[key] - val) <= 1e-12 * max(1e-300, abs(val)), (key, got[key], val)
