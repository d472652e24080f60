"""Pins of the oracle's nuclear gradient and of the basis normalisation (no GPU).

Gradient (dE_J/dR_A at fixed D(k), fixed pair list and fixed G set; the paper has
no forces, the derivative follows from eq. "cart gaussian function" and eq.
"AFT for pair density"): the oracle's analytic gradient -- the D-weighted centre
derivatives of every pair transform contracted with v(G) rho(-G) and assigned to
the atoms of shells a and b -- is checked against central finite differences of
the oracle's own G-space energy.  The finite differences touch none of that
assembly: they only call the energy with displaced atoms, after confirming that
the displaced geometry keeps exactly the same screened pair list (the gradient's
definition holds the list fixed).  A uniform translation leaves E_J unchanged,
so the atom gradients sum to zero.

Normalisation: every Cartesian component of a shell shares N(l, a), the factor
that normalises x^l e^{-a r^2}.  The self-overlap of component (lx, ly, lz) is
then prod_x Gamma(l_x + 1/2) / (Gamma(l + 1/2) Gamma(1/2)^2) (1D Gaussian
moments; 1 for x^l itself), checked against the oracle's transform at G = 0.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_16460_amd import synth

DELTA = 1e-4


def gradient_cases():
    # (name, problem): s..f shells, two or three atoms, Gamma and a k-mesh,
    # a non-orthogonal cell; exponents kept moderate so each energy costs ms
    return [
        ("sp_gamma", synth.small_problem(kind="g_sp", seed=301, kmesh=(1, 1, 1), lmax=1, natm=2, lo=0.3, hi=6.0)),
        ("spd_k211", synth.small_problem(kind="g_spd", seed=302, kmesh=(2, 1, 1), lmax=2, natm=3, lo=0.3, hi=5.0)),
        ("spdf_gamma", synth.small_problem(kind="g_spdf", seed=303, kmesh=(1, 1, 1), lmax=3, natm=2, lo=0.35,
                                           hi=4.0)),
    ]


def displaced(prob, atom, x, h):
    xyz = np.array(prob.xyz, dtype=np.float64, copy=True)
    xyz[atom, x] += h
    return prob.with_(xyz=xyz)


@pytest.mark.parametrize("name,prob", gradient_cases(), ids=[c[0] for c in gradient_cases()])
def test_gradient_matches_finite_differences(name, prob):
    D = synth.make_density(prob, 310)
    ref = O.build_j(prob, D, want_J=False, want_rho=False, want_grad=True)
    g = ref["grad"]
    base_pairs = O.pairs(prob)
    fd = np.zeros_like(g)
    for a in range(prob.natm):
        for x in range(3):
            e = []
            for h in (DELTA, -DELTA):
                pd = displaced(prob, a, x, h)
                # the gradient holds the pair list fixed: the displaced cell must keep it
                assert np.array_equal(O.pairs(pd), base_pairs), (name, a, x, h)
                e.append(O.build_j(pd, D, want_J=False, want_rho=False)["E_G"])
            fd[a, x] = (e[0] - e[1]) / (2 * DELTA)
    scale = np.max(np.abs(g))
    err = np.max(np.abs(fd - g))
    print(f"{name}: max|g|={scale:.3e} max|FD-g|={err:.3e}")
    # central differences: truncation ~ DELTA^2 E'''/6, rounding ~ 1e-16 E / DELTA
    assert err <= 1e-7 * scale
    # a uniform translation leaves E_J unchanged (G and -G cancel in the sum)
    assert np.max(np.abs(g.sum(axis=0))) <= 1e-11 * scale


def test_gradient_is_linear_in_each_density_weight():
    # dE/dR is quadratic in D: g[cD] = c^2 g[D], and g[D1 + D2] - g[D1] - g[D2] is
    # the symmetric cross term, equal to the derivative of <D1, J[D2]> (by
    # finite differences of the oracle's bilinear form, no gradient assembly)
    prob = synth.small_problem(kind="g_bil", seed=304, kmesh=(1, 1, 1), lmax=1, natm=2, lo=0.3, hi=5.0)
    D1 = synth.make_density(prob, 311)
    D2 = synth.make_density(prob, 312)
    g1 = O.build_j(prob, D1, want_J=False, want_rho=False, want_grad=True)["grad"]
    g2 = O.build_j(prob, D2, want_J=False, want_rho=False, want_grad=True)["grad"]
    g12 = O.build_j(prob, D1 + D2, want_J=False, want_rho=False, want_grad=True)["grad"]
    gc = O.build_j(prob, 1.7 * D1, want_J=False, want_rho=False, want_grad=True)["grad"]
    scale = np.max(np.abs(g12))
    assert np.max(np.abs(gc - 1.7 ** 2 * g1)) <= 1e-12 * np.max(np.abs(gc))
    cross = g12 - g1 - g2
    fd = np.zeros_like(cross)
    for a in range(prob.natm):
        for x in range(3):
            v = []
            for h in (DELTA, -DELTA):
                pd = displaced(prob, a, x, h)
                J2 = O.build_j(pd, D2, want_rho=False)["J"]
                # <D1, J[D2]> = sum_k w_k sum D1(k) J2(k); the cross term of E is twice half of it
                v.append(np.sum(D1 * J2).real / prob.nk)
            fd[a, x] = (v[0] - v[1]) / (2 * DELTA)
    assert np.max(np.abs(fd - cross)) <= 1e-7 * scale


def moment_ratio(c, l):
    """Self-overlap of the Cartesian component c = (lx, ly, lz) when its
    normalisation is the one of x^l (1D Gaussian moments: the exponent and the
    centre cancel)."""
    num = math.gamma(c[0] + 0.5) * math.gamma(c[1] + 0.5) * math.gamma(c[2] + 0.5)
    return num / (math.gamma(l + 0.5) * math.gamma(0.5) ** 2)


@pytest.mark.parametrize("l", [0, 1, 2, 3, 4])
def test_normalisation_self_overlap(l):
    rng = np.random.default_rng(320 + l)
    for _ in range(3):
        a = float(np.exp(rng.uniform(np.log(0.05), np.log(5e3))))
        R = rng.uniform(-3, 3, 3)
        S = O.pair_ft(l, l, a, R, a, R, np.zeros(3))
        comps = synth.cart_components(l)
        for i, c in enumerate(comps):
            ref = moment_ratio(c, l)
            assert abs(S[i, i] - ref) <= 1e-13, (l, c, S[i, i], ref)
        # x^l itself (the first component) is normalised
        assert abs(S[0, 0] - 1.0) <= 1e-13
