"""Pins of the per-pair reciprocal-space cut (section "Integral screening"; no GPU).

The cut radius of a pair block comes from its most compact primitive pair: the
largest |G| below the global cutoff where the screening objective
  eps(G) = 8 pi eta G (4 pi / G^2) e^{-G^2/4 omega^2} |F|_inf(G),
  eta = [1/(a_a + a_b) + 1/omega^2]^{-1}      (eqs. "AFT screening obj", "eta_munu")
still reaches the threshold eps_G.  Checked here:
  * the objective of an s-s pair against its closed form (Gaussian product
    theorem: |F| = N_a N_b (pi/p)^{3/2} K e^{-G^2/4p} in every direction);
  * the search: at the cut the objective is below eps_G, just inside it is not,
    and it stays below eps_G everywhere between the cut and the global cutoff
    (direct evaluations on a fine grid);
  * the definition with cuts stays within the threshold of the plain one: E_J,
    J(k) and V(G) = v rho(G) differ by ~1e-13 relative, and the three energy routes,
    rho(-G) = conj rho(G) and J Hermiticity still hold;
  * the library's host plan counts the pair-G work inside the cuts by per-line
    root finding of |G(n_u)|^2 = gc2 (eq. "G-space root finding"); the count
    equals a brute-force enumeration over the oracle's cut radii and G set.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_16460_amd import pwdf, synth


def test_ss_objective_closed_form():
    rng = np.random.default_rng(400)
    for _ in range(10):
        aa, ab = np.exp(rng.uniform(np.log(0.05), np.log(50.0), 2))
        A, B = rng.uniform(-2, 2, 3), rng.uniform(-2, 2, 3)
        omega = float(rng.uniform(0.3, 0.8))
        G = float(rng.uniform(0.2, 5.0))
        p = aa + ab
        K = math.exp(-aa * ab / p * np.sum((A - B) ** 2))
        F = synth.gto_norm(0, aa) * synth.gto_norm(0, ab) * (math.pi / p) ** 1.5 * K * math.exp(-G * G / (4 * p))
        eta = 1.0 / (1.0 / p + 1.0 / omega ** 2)
        ref = 8 * math.pi * eta * G * (4 * math.pi / G ** 2) * math.exp(-G * G / (4 * omega ** 2)) * F
        got, _ = O.pair_cut(0, 0, aa, A, ab, B, omega, 1e-12, G)
        assert abs(got - ref) <= 1e-13 * ref


@pytest.mark.parametrize("la,lb", [(0, 0), (1, 0), (2, 1), (3, 3)])
def test_cut_brackets_the_threshold(la, lb):
    rng = np.random.default_rng(410 + 4 * la + lb)
    eps = 1e-12
    for _ in range(4):
        aa, ab = np.exp(rng.uniform(np.log(0.05), np.log(30.0), 2))
        A = rng.uniform(-1, 1, 3)
        B = A + rng.uniform(-4, 4, 3)
        omega = float(rng.uniform(0.35, 0.6))
        gglob = 2 * omega * math.sqrt(-math.log(eps))
        _, cut = O.pair_cut(la, lb, aa, A, ab, B, omega, eps, 1.0)
        assert 0 < cut <= gglob
        obj = lambda G: O.pair_cut(la, lb, aa, A, ab, B, omega, eps, G)[0]  # noqa: E731
        if cut < gglob:
            assert obj(cut) < eps
            # (a pair whose objective stays below eps_G down to |G| ~ 1e-6 -- far
            # inside the shortest G vector of any cell -- sees no G at all; its
            # bisection ends near 0 at its resolution)
            if cut > 1e-6:
                assert obj(cut * (1 - 1e-9)) >= eps
        # below the threshold all the way out to the global cutoff
        for G in np.linspace(cut, gglob, 200)[1:]:
            assert obj(G) < eps, (la, lb, G, cut)


@pytest.mark.parametrize("name,prob", [
    ("cubic2_gamma", synth.config_problem(1)),
    ("spd_k221", synth.small_problem(kind="c1", seed=420, kmesh=(2, 2, 1), lmax=2, natm=2, lo=0.2, hi=6.0)),
    ("spdf_mixed", synth.small_problem(kind="c2", seed=421, kmesh=(1, 1, 1), lmax=3, natm=3, lo=0.1, hi=50.0)),
], ids=["cubic2_gamma", "spd_k221", "spdf_mixed"])
def test_cut_definition_within_threshold(name, prob):
    D = synth.make_density(prob, 430)
    full = O.build_j(prob, D)
    cut = O.build_j(prob, D, pair_gcut=1)
    E = full["E_G"]
    assert abs(cut["E_G"] - E) <= 1e-11 * E
    assert np.max(np.abs(cut["J"] - full["J"])) <= 1e-11 * np.max(np.abs(full["J"]))
    # rho itself loses the contributions the cut drops where the kernel has made
    # them negligible: the potential V = v rho is what must agree
    G2 = np.array([np.sum((prob_B(prob) @ m) ** 2) for m in full["miller"]])
    v = 4 * math.pi * np.exp(-G2 / (4 * prob.omega ** 2)) / G2
    assert np.array_equal(cut["miller"], full["miller"])
    assert np.max(np.abs(v * (cut["rho"] - full["rho"]))) <= 1e-11 * np.max(np.abs(v * full["rho"]))
    # structure is kept: energy routes, rho(-G) = conj rho(G), Hermitian J(k)
    assert abs(cut["E_real"] - cut["E_G"]) <= 1e-13 * E and abs(cut["E_k"] - cut["E_G"]) <= 1e-13 * E
    idx = {tuple(m): i for i, m in enumerate(cut["miller"])}
    mi = np.array([idx[tuple(-m)] for m in cut["miller"]])
    assert np.max(np.abs(cut["rho"][mi] - cut["rho"].conj())) <= 1e-14 * np.max(np.abs(cut["rho"]))
    J = cut["J"]
    assert np.max(np.abs(J - J.conj().transpose(0, 2, 1))) <= 1e-13 * np.max(np.abs(J))


def g2_of_set(prob):
    """|G|^2 of the oracle's G set (both G and -G), sorted."""
    full = O.build_j(prob, np.zeros((prob.nk, prob.nbf, prob.nbf), dtype=complex), want_J=False)
    return np.sort(np.array([np.sum((prob_B(prob) @ m) ** 2) for m in full["miller"]]))


def brute_force_pairG(prob, g2=None):
    """Sum over the unique pairs of the half-space G vectors inside the pair's cut
    (the oracle's cut radii; the oracle's G set, or the given |G|^2 of both G and -G)."""
    P = O.pairs(prob)
    g2 = g2_of_set(prob) if g2 is None else np.sort(g2)
    poff = prob.prim_offsets()
    blocks = {}
    for r in P:
        sa, sb, ia, ib = (int(x) for x in r[:4])
        la, lb = int(prob.shell_l[sa]), int(prob.shell_l[sb])
        if la < lb or (la == lb and sa > sb):
            continue  # the library keeps one of (a,b,L) ~ (b,a,-L)
        m = tuple(int(x) for x in r[4:])
        if sa == sb and m < (0, 0, 0) and any(m):
            continue
        blocks.setdefault((sa, sb, m), []).append((ia, ib))
    total = 0
    for (sa, sb, m), prims in blocks.items():
        la, lb = int(prob.shell_l[sa]), int(prob.shell_l[sb])
        ia, ib = max(prims, key=lambda t: prob.exps[t[0]] + prob.exps[t[1]])
        A = prob.xyz[prob.shell_atom[sa]]
        B = prob.xyz[prob.shell_atom[sb]] + np.array(m) @ prob.lattice
        _, c = O.pair_cut(la, lb, prob.exps[ia], A, prob.exps[ib], B, prob.omega, prob.eps_G, 1.0)
        total += len(prims) * int(np.searchsorted(g2, c * c, side="right")) // 2
    del poff
    return total


def prob_B(prob):
    return 2 * math.pi * np.linalg.inv(prob.lattice)  # columns b_i


@pytest.mark.parametrize("name,prob", [
    ("cubic2_gamma", synth.config_problem(1)),
    ("spdf_mixed", synth.small_problem(kind="c3", seed=440, kmesh=(2, 1, 1), lmax=3, natm=3, lo=0.1, hi=40.0)),
], ids=["cubic2_gamma", "spdf_mixed"])
def test_plan_root_finding_count_matches_brute_force(name, prob):
    got = pwdf.plan_stats(prob.with_(pair_gcut=1))["pairG_evals"] / 2
    ref = brute_force_pairG(prob)
    full = pwdf.plan_stats(prob)["pairG_evals"] / 2
    print(f"{name}: pair-G per pass inside the cuts {got:.0f} (brute force {ref}), without cuts {full:.0f}")
    assert got < full
    # the two implementations place each cut radius within ~1e-12 of each other: a
    # G vector on the boundary may land on either side
    assert abs(got - ref) <= 1e-6 * ref


@pytest.mark.parametrize("name,prob", [
    ("cubic2_gamma", synth.config_problem(1)),
    ("spdf_mixed", synth.small_problem(kind="c3", seed=440, kmesh=(2, 1, 1), lmax=3, natm=3, lo=0.1, hi=40.0)),
], ids=["cubic2_gamma", "spdf_mixed"])
def test_plan_head_of_the_G_set(name, prob):
    """The head of the G set (contracted with FP64 tiles in the FP32-MFMA form):
    the G with v(G) >= 2^-20 max v (the default head weight), v = 4 pi
    e^{-G^2/4 omega^2} / G^2; its pair-G work with and without per-pair cuts
    against brute force."""
    g2 = g2_of_set(prob)
    v = np.exp(-g2 / (4 * prob.omega ** 2)) / g2
    head = g2[v >= v.max() / 1048576.0]
    st = pwdf.plan_stats(prob)
    assert st["nG_head"] == len(head) // 2 and 0 < st["nG_head"] < st["nG"] // 2
    assert st["pairG_head"] == 2 * st["npairs"] * st["nG_head"]
    sc = pwdf.plan_stats(prob.with_(pair_gcut=1))
    ref = brute_force_pairG(prob, head)
    print(f"{name}: head {st['nG_head']} of {st['nG'] // 2} G; pair-G on the head with cuts {sc['pairG_head'] / 2:.0f}"
          f" (brute force {ref}), without {st['pairG_head'] / 2:.0f}")
    assert abs(sc["pairG_head"] / 2 - ref) <= 1e-6 * ref
