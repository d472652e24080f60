"""Pins of the oracle's compact/diffuse classification (no GPU).

Section "Density classification: compact and diffuse", eq. "cd cutoff": a
primitive is diffuse when its exponent lies below alpha_cut = w^2/2; a pair of
two diffuse primitives (DD) is taken with the full-range kernel 4 pi/G^2 against
everything, while compact pairs (CC, CD) keep the long-range kernel among
themselves.  Pins, each against something the oracle does not compute itself:

  * real space: classification adds, for every interaction with a DD side, the
    short-range part erfc(w r)/r that the long-range kernel leaves out.  For s
    Gaussians at the Gamma point that part is a closed-form lattice sum of
    Gaussian-charge interactions,
        q_i q_j [erf(sqrt(mu) R) - erf(sqrt(nu) R)] / R,
        mu = p_i p_j / (p_i + p_j),  1/nu = 1/mu + 1/w^2,
    minus the G = 0 term pi Q_a Q_b / (w^2 Omega) of its Fourier series (the G
    set excludes G = 0).  So
        E_cls - E_lr = RS(C, D) + RS(D, D)/2 - pi (2 Q_C Q_D + Q_D^2) / (2 w^2 Omega)
    with RS(X, Y) = sum_{i in X, j in Y, T} q_i q_j I(|P_i - P_j - T|), on the
    oracle's own pair list (the screened list is part of the definition); the
    pair charges q = D N_a N_b K (pi/p)^{3/2} come from the Gaussian product
    rule, written out here.
  * the three energy routes (real space 1/2 sum D J, G space, k space) agree:
    a DD pair contracted with the compact pairs' potential, or the other way
    round, breaks the agreement;
  * no diffuse primitive: the classified oracle is the unclassified one, bit for
    bit;
  * the analytic gradient with classification matches central differences of the
    classified energy.
"""
import math

import numpy as np
import pytest
from scipy.special import erf

from oracle import oracle as O
from paper_2509_16460_amd import synth

DELTA = 1e-4


def s_problem(exps, omega, natm=2):
    lat = np.array([[5.0, 0.0, 0.0], [0.4, 5.3, 0.0], [-0.3, 0.2, 4.8]])
    xyz = np.array([[0.1, 0.2, 0.3], [2.6, 2.4, 2.2]])[:natm]
    return synth.build_problem("cd_s", lat, xyz, [0] * natm, {0: [np.asarray(exps, dtype=float)]}, (1, 1, 1),
                               omega, eps_G=1e-14, nelec=2.0 * natm)


def pair_charges(prob, D):
    """Centres P, exponents p and charges q of the oracle's primitive pairs (s shells)."""
    pl = O.pairs(prob)
    lat = np.asarray(prob.lattice)
    xyz = np.asarray(prob.xyz)
    ex = np.asarray(prob.exps)
    sa, sb, ia, ib = pl[:, 0], pl[:, 1], pl[:, 2], pl[:, 3]
    L = pl[:, 4:7] @ lat
    A = xyz[prob.shell_atom[sa]]
    B = xyz[prob.shell_atom[sb]] + L
    a, b = ex[ia], ex[ib]
    p = a + b
    P = (a[:, None] * A + b[:, None] * B) / p[:, None]
    K = np.exp(-a * b / p * np.sum((A - B) ** 2, axis=1))
    N = lambda x: (2 * x / math.pi) ** 0.75  # noqa: E731  (s normalisation)
    q = D[0].real[sa, sb] * N(a) * N(b) * K * (math.pi / p) ** 1.5
    return P, p, q, a, b


def rs_sum(Pi, pi, qi, Pj, pj, qj, lat, omega, nT=3):
    """sum_{i, j, T} q_i q_j [erf(sqrt(mu) R) - erf(sqrt(nu) R)] / R, R = |P_i - P_j - T|."""
    ms = np.array(np.meshgrid(*[np.arange(-nT, nT + 1)] * 3, indexing="ij")).reshape(3, -1).T
    T = ms @ lat
    tot = 0.0
    for i in range(len(qi)):
        mu = pi[i] * pj / (pi[i] + pj)
        nu = 1.0 / (1.0 / mu + 1.0 / omega ** 2)
        d = Pi[i][None, None, :] - Pj[:, None, :] - T[None, :, :]
        R = np.linalg.norm(d, axis=2)
        sm, sn = np.sqrt(mu)[:, None], np.sqrt(nu)[:, None]
        with np.errstate(invalid="ignore", divide="ignore"):
            f = (erf(sm * R) - erf(sn * R)) / R
        f = np.where(R < 1e-12, 2.0 * (sm - sn) / math.sqrt(math.pi) + 0.0 * R, f)
        tot += qi[i] * np.sum(qj[:, None] * f)
    return tot


@pytest.mark.parametrize("exps", [[0.35, 2.0], [0.45]], ids=["mixed", "all_diffuse"])
def test_short_range_difference_in_real_space(exps):
    omega = 1.0
    ac = omega ** 2 / 2
    prob = s_problem(exps, omega)
    D = synth.make_density(prob, 41)
    e_lr = O.build_j(prob, D, want_J=False, want_rho=False)["E_G"]
    e_cls = O.build_j(prob, D, want_J=False, want_rho=False, alpha_cut=ac)["E_G"]
    P, p, q, a, b = pair_charges(prob, D)
    dd = (a < ac) & (b < ac)
    lat = np.asarray(prob.lattice)
    Omega = abs(np.linalg.det(lat))
    C, Dm = ~dd, dd
    assert Dm.sum() > 0
    rs_cd = rs_sum(P[C], p[C], q[C], P[Dm], p[Dm], q[Dm], lat, omega) if C.any() else 0.0
    rs_dd = rs_sum(P[Dm], p[Dm], q[Dm], P[Dm], p[Dm], q[Dm], lat, omega)
    QC, QD = q[C].sum(), q[Dm].sum()
    expect = rs_cd + 0.5 * rs_dd - math.pi * (2 * QC * QD + QD ** 2) / (2 * omega ** 2 * Omega)
    got = e_cls - e_lr
    print(f"E_lr={e_lr:.12f} E_cls={e_cls:.12f} diff={got:.12e} real-space={expect:.12e}")
    assert abs(got) > 1e-3  # the classification changes the energy
    assert abs(got - expect) <= 1e-10 * max(1.0, abs(e_cls))


def cd_problem(kmesh=(2, 1, 1), lmax=2, natm=2, seed=61, r_max=0.0):
    """s, p (and d) shells with one diffuse and one compact exponent each against
    alpha_cut = w^2/2 = 0.125 (w = 0.5), so CC, CD and DD pairs all occur; a
    non-orthogonal cell."""
    rng = np.random.default_rng(seed)
    lat = np.array([[4.2, 0.0, 0.0], [0.3, 4.6, 0.0], [-0.4, 0.5, 3.9]])
    xyz = rng.uniform(0, 1, size=(natm, 3)) @ lat
    ex = {0: [np.array(e) for e in ([2.2, 0.09], [1.3, 0.1], [0.9, 0.11])[:lmax + 1]]}
    prob = synth.build_problem("cd", lat, xyz, [0] * natm, ex, kmesh, 0.5, nelec=2.0 * natm, seed=seed,
                               r_max=r_max)
    return prob.with_(alpha_cut=0.125)


@pytest.fixture(scope="module")
def cd_case():
    prob = cd_problem()
    D = synth.make_density(prob, 62)
    return prob, D, O.build_j(prob, D)


def test_cd_case_has_every_pair_class(cd_case):
    prob, _, _ = cd_case
    ex = np.asarray(prob.exps)
    assert (ex < prob.alpha_cut).sum() >= 2 and (ex > prob.alpha_cut).sum() >= 2


def test_energy_routes_agree_with_classification(cd_case):
    prob, D, r = cd_case
    e = r["E_G"]
    assert abs(r["E_real"] - e) <= 1e-12 * abs(e)
    assert abs(r["E_k"] - e) <= 1e-12 * abs(e)
    J = r["J"]
    assert np.max(np.abs(J - np.conj(np.transpose(J, (0, 2, 1))))) <= 1e-12 * np.max(np.abs(J))
    assert r["maxImJ"] <= 1e-12 * r["maxJ"]
    ru = O.build_j(prob, D, alpha_cut=0.0, want_rho=False)
    assert abs(ru["E_G"] - e) > 1e-6 * abs(e)  # the classification is not a no-op here


def test_no_diffuse_primitive_is_unclassified():
    prob = synth.small_problem(kind="cd0", seed=63, kmesh=(2, 1, 1), lmax=1, natm=2, lo=0.3, hi=5.0)
    D = synth.make_density(prob, 64)
    # one thread: the real-space energy is an OpenMP reduction
    a = O.build_j(prob, D, nthreads=1)
    b = O.build_j(prob, D, alpha_cut=0.1, nthreads=1)
    assert a["E_G"] == b["E_G"] and a["E_real"] == b["E_real"]
    assert np.array_equal(a["J"], b["J"]) and np.array_equal(a["rho"], b["rho"])


def test_gradient_with_classification_matches_finite_differences():
    # centre distances capped at 10 Bohr (a shorter pair list; each energy is a
    # full oracle call)
    prob = cd_problem(kmesh=(1, 1, 1), lmax=1, seed=65, r_max=10.0)
    assert (np.asarray(prob.exps) < prob.alpha_cut).sum() >= 2
    D = synth.make_density(prob, 66)
    g = O.build_j(prob, D, want_J=False, want_rho=False, want_grad=True)["grad"]
    base = O.pairs(prob)
    fd = np.zeros_like(g)
    for at in range(prob.natm):
        for x in range(3):
            e = []
            for h in (DELTA, -DELTA):
                xyz = np.array(prob.xyz, copy=True)
                xyz[at, x] += h
                pd = prob.with_(xyz=xyz)
                assert np.array_equal(O.pairs(pd), base)
                e.append(O.build_j(pd, D, want_J=False, want_rho=False)["E_G"])
            fd[at, x] = (e[0] - e[1]) / (2 * DELTA)
    scale = np.max(np.abs(g))
    print(f"max|g|={scale:.3e} max|FD-g|={np.max(np.abs(fd - g)):.3e}")
    assert np.max(np.abs(fd - g)) <= 1e-7 * scale
    assert np.max(np.abs(g.sum(axis=0))) <= 1e-11 * scale
