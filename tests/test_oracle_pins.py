"""Pins of the FP64 oracle against facts fixed by the mathematics, not by the
oracle's own formulas (no GPU).

Pair transform (eq. "AFT for pair density", evaluated through the Gaussian
product theorem and the Hermite-polynomial transform):
  * 1D numerical quadrature of every axis factor, including l up to (4,3);
  * the s-s closed form (Gaussian product theorem + transform of a Gaussian);
  * G = 0 against an Obara-Saika overlap recurrence (different algebra);
  * translation: F(A+d, B+d) = e^{-iG.d} F(A, B);
  * centre derivatives: central finite differences, and (dA + dB) F = -iG F;
  * the McMurchie-Davidson Hermite-expansion route (different algebra).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_16460_amd import synth


def quad_axis(i, j, aa, Ax, ab, Bx, G):
    """Trapezoid rule on a fine uniform grid (spectrally accurate for this integrand)."""
    p = aa + ab
    P = (aa * Ax + ab * Bx) / p
    w = 1.0 / math.sqrt(p)
    x = np.linspace(P - 14 * w, P + 14 * w, 8001)
    h = x[1] - x[0]
    f = (x - Ax) ** i * (x - Bx) ** j * np.exp(-aa * (x - Ax) ** 2 - ab * (x - Bx) ** 2) * np.exp(-1j * G * x)
    scale = h * np.sum(np.abs(f))
    return h * (np.sum(f) - 0.5 * (f[0] + f[-1])), scale


@pytest.mark.parametrize("i,j", [(i, j) for i in range(5) for j in range(4)])
def test_axis_factor_matches_quadrature(i, j):
    rng = np.random.default_rng(100 + 10 * i + j)
    for _ in range(6):
        aa, ab = np.exp(rng.uniform(np.log(0.1), np.log(20.0), 2))
        Ax, Bx = rng.uniform(-3, 3, 2)
        G = rng.uniform(-6, 6)
        got = O.ft_axis(i, j, aa, Ax, ab, Bx, G)
        ref, scale = quad_axis(i, j, aa, Ax, ab, Bx, G)
        assert abs(got - ref) <= 1e-12 * max(scale, 1e-300), (i, j, got, ref, scale)


def test_ss_closed_form():
    rng = np.random.default_rng(7)
    for _ in range(20):
        aa, ab = np.exp(rng.uniform(np.log(0.05), np.log(1e3), 2))
        A, B, G = rng.uniform(-4, 4, 3), rng.uniform(-4, 4, 3), rng.uniform(-5, 5, 3)
        p = aa + ab
        P = (aa * A + ab * B) / p
        K = math.exp(-aa * ab / p * np.sum((A - B) ** 2))
        N = synth.gto_norm(0, aa) * synth.gto_norm(0, ab)
        ref = N * (math.pi / p) ** 1.5 * K * math.exp(-G @ G / (4 * p)) * np.exp(-1j * G @ P)
        got = O.pair_ft(0, 0, aa, A, ab, B, G)[0, 0]
        assert abs(got - ref) <= 1e-14 * abs(N * (math.pi / p) ** 1.5) + 1e-300


@pytest.mark.parametrize("la,lb", [(la, lb) for la in range(4) for lb in range(4)])
def test_G0_equals_obara_saika_overlap(la, lb):
    rng = np.random.default_rng(200 + 4 * la + lb)
    aa, ab = np.exp(rng.uniform(np.log(0.1), np.log(30.0), 2))
    A, B = rng.uniform(-1.5, 1.5, 3), rng.uniform(-1.5, 1.5, 3)
    p = aa + ab
    mu = aa * ab / p
    P = (aa * A + ab * B) / p
    tabs = []
    for x in range(3):
        s00 = math.sqrt(math.pi / p) * math.exp(-mu * (A[x] - B[x]) ** 2)
        tabs.append(synth._os_overlap_1d(la, lb, p, P[x] - A[x], P[x] - B[x], s00))
    N = synth.gto_norm(la, aa) * synth.gto_norm(lb, ab)
    got = O.pair_ft(la, lb, aa, A, ab, B, np.zeros(3))
    for ia, (ax, ay, az) in enumerate(synth.cart_components(la)):
        for ib, (bx, by, bz) in enumerate(synth.cart_components(lb)):
            ref = N * tabs[0][ax][bx] * tabs[1][ay][by] * tabs[2][az][bz]
            assert abs(got[ia, ib] - ref) <= 1e-13 * max(1.0, abs(ref)), (ia, ib)


def test_translation_phase():
    rng = np.random.default_rng(3)
    for la, lb in [(1, 0), (2, 1), (3, 3), (2, 2)]:
        aa, ab = 0.7, 2.3
        A, B, G, d = rng.uniform(-2, 2, 3), rng.uniform(-2, 2, 3), rng.uniform(-3, 3, 3), rng.uniform(-5, 5, 3)
        F0 = O.pair_ft(la, lb, aa, A, ab, B, G)
        F1 = O.pair_ft(la, lb, aa, A + d, ab, B + d, G)
        assert np.max(np.abs(F1 - np.exp(-1j * G @ d) * F0)) <= 1e-13 * np.max(np.abs(F0))


@pytest.mark.parametrize("la,lb", [(0, 0), (1, 0), (1, 1), (2, 1), (3, 2), (3, 3)])
def test_centre_derivatives(la, lb):
    rng = np.random.default_rng(40 + la * 4 + lb)
    aa, ab = 0.9, 1.7
    A, B, G = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3), rng.uniform(-3, 3, 3)
    F, dA, dB = O.pair_ft(la, lb, aa, A, ab, B, G, deriv=True)
    # translation generator: (dA + dB) F = -iG F
    for x in range(3):
        assert np.max(np.abs(dA[x] + dB[x] + 1j * G[x] * F)) <= 1e-12 * max(1.0, np.max(np.abs(F)))
    # central differences, step 1e-4 (truncation ~1e-8 relative)
    h = 1e-4
    for x in range(3):
        e = np.zeros(3)
        e[x] = h
        fd = (O.pair_ft(la, lb, aa, A + e, ab, B, G) - O.pair_ft(la, lb, aa, A - e, ab, B, G)) / (2 * h)
        assert np.max(np.abs(fd - dA[x])) <= 1e-7 * max(1.0, np.max(np.abs(dA[x])))
        fd = (O.pair_ft(la, lb, aa, A, ab, B + e, G) - O.pair_ft(la, lb, aa, A, ab, B - e, G)) / (2 * h)
        assert np.max(np.abs(fd - dB[x])) <= 1e-7 * max(1.0, np.max(np.abs(dB[x])))


def md_block(la, lb, aa, A, ab, B, G):
    """McMurchie-Davidson route: x_A^i x_B^j e^{..} = K sum_t E_t d^t/dP^t e^{-p x_P^2};
    transform of the t-th derivative is (-iG)^t sqrt(pi/p) e^{-G^2/4p} e^{-iGP}."""
    p = aa + ab
    P = (aa * A + ab * B) / p
    K = math.exp(-aa * ab / p * np.sum((A - B) ** 2))
    E = []
    for x in range(3):
        XPA, XPB = P[x] - A[x], P[x] - B[x]
        T = np.zeros((la + 1, lb + 1, la + lb + 2))
        T[0, 0, 0] = 1.0
        for i in range(la + 1):
            for j in range(lb + 1):
                if i == 0 and j == 0:
                    continue
                for t in range(i + j + 1):
                    if i > 0:
                        v = XPA * T[i - 1, j, t] + (t + 1) * T[i - 1, j, t + 1]
                        if t > 0:
                            v += T[i - 1, j, t - 1] / (2 * p)
                    else:
                        v = XPB * T[i, j - 1, t] + (t + 1) * T[i, j - 1, t + 1]
                        if t > 0:
                            v += T[i, j - 1, t - 1] / (2 * p)
                    T[i, j, t] = v
        E.append(T)
    base = (math.pi / p) ** 1.5 * K * math.exp(-G @ G / (4 * p)) * np.exp(-1j * G @ P)
    N = synth.gto_norm(la, aa) * synth.gto_norm(lb, ab)
    ca, cb = synth.cart_components(la), synth.cart_components(lb)
    out = np.zeros((len(ca), len(cb)), dtype=complex)
    for ia, a in enumerate(ca):
        for ib, b in enumerate(cb):
            val = 1.0 + 0j
            for x in range(3):
                val *= sum(E[x][a[x], b[x], t] * (-1j * G[x]) ** t for t in range(a[x] + b[x] + 1))
            out[ia, ib] = N * base * val
    return out


@pytest.mark.parametrize("la,lb", [(la, lb) for la in range(4) for lb in range(la + 1)])
def test_hermite_expansion_route(la, lb):
    rng = np.random.default_rng(60 + la * 4 + lb)
    for _ in range(3):
        aa, ab = np.exp(rng.uniform(np.log(0.08), np.log(5e3), 2))
        A, B, G = rng.uniform(-3, 3, 3), rng.uniform(-3, 3, 3), rng.uniform(-5, 5, 3)
        got = O.pair_ft(la, lb, aa, A, ab, B, G)
        ref = md_block(la, lb, aa, A, ab, B, G)
        scale = synth.gto_norm(la, aa) * synth.gto_norm(lb, ab) * (math.pi / (aa + ab)) ** 1.5 * \
            (1.0 + np.max(np.abs(G)) + 1 / math.sqrt(aa + ab) + np.max(np.abs(A - B))) ** (la + lb)
        assert np.max(np.abs(got - ref)) <= 1e-13 * scale
