"""System-level pins of the FP64 oracle (no GPU).

Each test checks the oracle against something it does not compute itself:
  * structure: rho(-G) = conj rho(G); J(k) Hermitian; E_J >= 0; the three energy
    routes agree; Omega rho(0) equals the electron count that the input
    generator fixed with its own overlap; E[cD] = c^2 E; <D1, J[D2]> symmetric;
  * translation of every atom leaves E_J and J unchanged and multiplies rho(G)
    by e^{-iG.d};
  * a unimodular change of lattice basis leaves E_J unchanged;
  * a 3x1x1 k-mesh equals the Gamma point of the 3x1x1 supercell (image and
    phase bookkeeping, sign conventions of D(L) and J(k));
  * a single compact Gaussian charge per cell reproduces an Ewald lattice sum
    whose total is independent of the splitting parameter (v(G), Omega, G != 0);
  * rho(G) from sampling the Bloch-sum density on a real-space grid + FFT.
"""
import math

import numpy as np
import pytest
from scipy.special import erfc

from oracle import oracle as O
from paper_2509_16460_amd import synth


@pytest.fixture(scope="module")
def small_k():
    prob = synth.small_problem(kind="spd", seed=5, kmesh=(2, 2, 1), lmax=2, natm=2, lo=0.2, hi=6.0)
    D = synth.make_density(prob, 77)
    return prob, D, O.build_j(prob, D)


def g_index(miller):
    return {tuple(m): i for i, m in enumerate(miller)}


def test_structure_invariants(small_k):
    prob, D, r = small_k
    rho, idx = r["rho"], g_index(r["miller"])
    mi = np.array([idx[tuple(-m)] for m in r["miller"]])
    assert np.max(np.abs(rho[mi] - rho.conj())) <= 1e-14 * np.max(np.abs(rho))
    J = r["J"]
    assert np.max(np.abs(J - J.conj().transpose(0, 2, 1))) <= 1e-13 * np.max(np.abs(J))
    E = r["E_G"]
    assert E > 0
    assert abs(r["E_real"] - E) <= 1e-13 * E and abs(r["E_k"] - E) <= 1e-13 * E
    assert r["maxImJ"] <= 1e-13 * r["maxJ"]
    # the generator scaled D with its own overlap over a slightly longer image list
    assert abs(r["charge"] - prob.nelec) <= 1e-10 * prob.nelec


def test_quadratic_and_bilinear(small_k):
    prob, D, r = small_k
    r2 = O.build_j(prob, 2.5 * D, want_rho=False)
    assert abs(r2["E_G"] - 6.25 * r["E_G"]) <= 1e-13 * r2["E_G"]
    assert np.max(np.abs(r2["J"] - 2.5 * r["J"])) <= 1e-13 * np.max(np.abs(r2["J"]))
    D2 = synth.make_density(prob, 78)
    rb = O.build_j(prob, D2, want_rho=False)
    a = np.sum(D * rb["J"]).real
    b = np.sum(D2 * r["J"]).real
    assert abs(a - b) <= 1e-12 * abs(a)


def test_translation_invariance(small_k):
    prob, D, r = small_k
    d = np.array([0.37, -1.21, 2.9])
    r2 = O.build_j(prob.with_(xyz=prob.xyz + d), D)
    assert abs(r2["E_G"] - r["E_G"]) <= 1e-13 * r["E_G"]
    assert np.max(np.abs(r2["J"] - r["J"])) <= 1e-13 * np.max(np.abs(r["J"]))
    # rho(G) e^{+iG.d} unchanged; G = B n
    B = 2 * math.pi * np.linalg.inv(prob.lattice)
    G = r["miller"] @ B.T
    assert np.max(np.abs(r2["rho"] * np.exp(1j * G @ d) - r["rho"])) <= 1e-13 * np.max(np.abs(r["rho"]))


def test_lattice_basis_change():
    prob = synth.small_problem(kind="sp", seed=8, lmax=1, natm=2)
    D = synth.make_density(prob, 81)
    r = O.build_j(prob, D, want_J=False)
    lat = prob.lattice.copy()
    lat2 = np.array([lat[0], lat[1] + lat[0], lat[2] - lat[1]])  # unimodular change
    r2 = O.build_j(prob.with_(lattice=lat2), D, want_J=False)
    assert r2["nG"] == r["nG"]
    assert abs(r2["E_G"] - r["E_G"]) <= 1e-12 * r["E_G"]


def test_kmesh_equals_supercell_gamma():
    prob = synth.small_problem(kind="sp", seed=9, kmesh=(3, 1, 1), lmax=1, natm=2, lo=0.3, hi=5.0)
    Dk = synth.make_density(prob, 91)
    rk = O.build_j(prob, Dk)
    nk = 3
    nbf = prob.nbf
    # D(L) for L = t a1 (t = 0,1,2 mod 3), D(L) = sum_k w_k e^{ik.L} D(k)
    kf = prob.kpoints_frac()
    DL = [sum(np.exp(2j * math.pi * kf[k, 0] * t) * Dk[k] for k in range(nk)) / nk for t in range(3)]
    assert max(np.max(np.abs(x.imag)) for x in DL) <= 1e-13
    sup = prob.with_(lattice=np.array([3 * prob.lattice[0], prob.lattice[1], prob.lattice[2]]),
                     xyz=np.vstack([prob.xyz + t * prob.lattice[0] for t in range(3)]),
                     shell_atom=np.concatenate([prob.shell_atom + t * prob.natm for t in range(3)]),
                     shell_l=np.tile(prob.shell_l, 3), shell_nprim=np.tile(prob.shell_nprim, 3),
                     exps=np.tile(prob.exps, 3), coefs=np.tile(prob.coefs, 3), kmesh=(1, 1, 1))
    Ds = np.zeros((1, 3 * nbf, 3 * nbf), dtype=complex)
    for t1 in range(3):
        for t2 in range(3):
            Ds[0, t1 * nbf:(t1 + 1) * nbf, t2 * nbf:(t2 + 1) * nbf] = DL[(t2 - t1) % 3].real
    rs = O.build_j(sup, Ds)
    assert abs(rs["E_G"] - nk * rk["E_G"]) <= 1e-12 * rs["E_G"]
    # J_super[(mu,0),(nu,t)] = sum_{L = t a1 mod 3 a1} J(L) = (1/Nk) sum_k e^{-ik.t a1} J(k)
    for t in range(3):
        JB = sum(np.exp(-2j * math.pi * kf[k, 0] * t) * rk["J"][k] for k in range(nk)) / nk
        blk = rs["J"][0, 0:nbf, t * nbf:(t + 1) * nbf]
        assert np.max(np.abs(blk - JB)) <= 1e-12 * np.max(np.abs(JB))


def test_ewald_splitting_independence():
    """One normalised compact s Gaussian per cell, D = q: rho(G) = (q/Omega) e^{-G^2/4a}
    ... gives E(w) = (q^2/2)(4 pi/Omega) sum_{G!=0} e^{-G^2/4 eta^2}/G^2 with
    1/eta^2 = 1/w^2 + 1/alpha.  The Ewald total
      Phi = (4pi/Omega) sum_G e^{-G^2/4eta^2}/G^2 + sum_{T!=0} erfc(eta T)/T
            - 2 eta/sqrt(pi) - pi/(Omega eta^2)
    is the Madelung potential of a neutralised point lattice, independent of eta."""
    lat = np.array([[4.0, 0.3, 0.0], [0.0, 4.4, 0.2], [0.5, 0.0, 3.7]])
    alpha = 2.0e3
    q = 1.3
    vals = []
    for w in (0.45, 0.8):
        prob = synth.build_problem("ewald", lat, [[0.1, 0.2, 0.3]], [0], {0: [np.array([alpha])]},
                                   (1, 1, 1), w, eps_G=1e-17)
        r = O.build_j(prob, np.full((1, 1, 1), q, dtype=complex), want_J=False)
        eta = 1.0 / math.sqrt(1.0 / w ** 2 + 1.0 / alpha)
        Omega = abs(np.linalg.det(lat))
        ms = np.array(np.meshgrid(*[np.arange(-12, 13)] * 3, indexing="ij")).reshape(3, -1).T
        T = np.linalg.norm(ms @ lat, axis=1)
        T = T[T > 0]
        real = np.sum(erfc(eta * T) / T)
        phi = 2 * r["E_G"] / q ** 2 + real - 2 * eta / math.sqrt(math.pi) - math.pi / (Omega * eta ** 2)
        vals.append(phi)
    assert abs(vals[0] - vals[1]) <= 1e-12 * abs(vals[0]), vals


def test_rho_from_realspace_grid_fft():
    """rho(r) = sum_k w_k sum_{mu nu} D_mu,nu(k) conj(chi^k_mu(r)) chi^k_nu(r),
    chi^k_nu(r) = sum_L e^{ik.L} phi_nu(r - L), sampled on an N^3 grid of the
    cell; rho(G) = (1/N^3) sum_r rho(r) e^{-iG.r}."""
    lat = np.array([[3.6, 0.0, 0.0], [0.4, 3.9, 0.0], [-0.3, 0.2, 3.4]])
    rng = np.random.default_rng(12)
    exps = {0: [np.array([1.4, 0.5]), np.array([0.9])]}
    xyz = rng.uniform(0, 1, (2, 3)) @ lat
    prob = synth.build_problem("grid", lat, xyz, [0, 0], exps, (3, 1, 1), 0.6, eps_pair=1e-22)
    D = synth.make_density(prob, 5)
    r = O.build_j(prob, D, want_J=False)
    N = 40
    f = (np.arange(N) / N)
    fr = np.array(np.meshgrid(f, f, f, indexing="ij")).reshape(3, -1).T
    rr = fr @ lat
    kf = prob.kpoints_frac()
    off = prob.shell_offsets()
    chis = np.zeros((prob.nk, prob.nbf, len(rr)), dtype=complex)
    ms = np.array(np.meshgrid(*[np.arange(-4, 5)] * 3, indexing="ij")).reshape(3, -1).T
    for s in range(prob.nshell):
        l = int(prob.shell_l[s])
        a = prob.exps[s]
        Nl = synth.gto_norm(l, a)
        for m in ms:
            d = rr - xyz[prob.shell_atom[s]] - m @ lat
            g = np.exp(-a * np.sum(d * d, axis=1))
            if g.max() < 1e-20:
                continue
            ph = np.exp(2j * math.pi * kf @ m)
            for c, (lx, ly, lz) in enumerate(synth.cart_components(l)):
                val = Nl * d[:, 0] ** lx * d[:, 1] ** ly * d[:, 2] ** lz * g
                chis[:, off[s] + c, :] += ph[:, None] * val[None, :]
    rho_r = np.zeros(len(rr))
    for k in range(prob.nk):
        rho_r += np.einsum("mn,mr,nr->r", D[k], chis[k].conj(), chis[k]).real / prob.nk
    B = 2 * math.pi * np.linalg.inv(lat)
    G = r["miller"] @ B.T
    sel = np.arange(0, len(G), max(1, len(G) // 60))
    ref = np.array([np.sum(rho_r * np.exp(-1j * rr @ G[i])) / N ** 3 for i in sel])
    assert np.max(np.abs(ref - r["rho"][sel])) <= 1e-10 * np.max(np.abs(r["rho"]))
