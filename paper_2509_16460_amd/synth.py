"""Seeded synthetic inputs: periodic cells, uncontracted Cartesian Gaussian basis
sets and density matrices D(k).

This module is shared by the HIP path's tests/benchmark and by the CPU oracle.  It
holds none of the long-range Coulomb arithmetic: it only draws geometries,
exponents and random positive semidefinite densities.  The one integral it
evaluates is the overlap S(k) (Obara-Saika recurrence), used solely to scale
each density so that sum_k w_k Tr(D(k) S(k)) equals the requested electron
count.

Conventions shared with the C ABI:
  * lattice: 3x3 row-major, rows are a1, a2, a3 (Bohr).
  * Cartesian components of a shell of angular momentum l are ordered by
    descending lexicographic (lx, ly, lz): x, y, z; xx, xy, xz, yy, yz, zz; ...
  * every component of a primitive shell carries the normalisation
    N(l, a) = (2a/pi)^(3/4) (4a)^(l/2) / sqrt((2l-1)!!) that normalises x^l e^{-a r^2}.
  * k-points of a Gamma-centred n1 x n2 x n3 mesh: k = sum_i (m_i / n_i) b_i with
    m_i = 0..n_i-1, flattened row-major over (m1, m2, m3); weight 1/N_k.
  * D(L) = sum_k w_k e^{i k.L} D(k) pairs phi_mu in cell 0 with phi_nu in cell L;
    J(k) = sum_L e^{i k.L} J(L).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def cart_components(l: int):
    """(lx, ly, lz) triples in descending lexicographic order."""
    out = []
    for lx in range(l, -1, -1):
        for ly in range(l - lx, -1, -1):
            out.append((lx, ly, l - lx - ly))
    return out


def _dfact(n: int) -> float:
    r = 1.0
    while n > 1:
        r *= n
        n -= 2
    return r


def gto_norm(l: int, a: float) -> float:
    return (2.0 * a / math.pi) ** 0.75 * (4.0 * a) ** (0.5 * l) / math.sqrt(_dfact(2 * l - 1))


@dataclasses.dataclass
class Problem:
    """One periodic system: cell, atoms, basis shells, k-mesh and range separation."""

    name: str
    lattice: np.ndarray          # (3,3) rows a1,a2,a3
    xyz: np.ndarray              # (natm,3)
    shell_atom: np.ndarray       # (nshell,) int32
    shell_l: np.ndarray          # (nshell,) int32
    shell_nprim: np.ndarray      # (nshell,) int32
    exps: np.ndarray             # (sum nprim,)
    coefs: np.ndarray            # (sum nprim,)
    kmesh: tuple                 # (n1,n2,n3)
    omega: float
    eps_pair: float = 1e-12
    eps_G: float = 1e-12
    r_max: float = 0.0
    nelec: float = 2.0
    seed: int = 0
    pair_gcut: int = 0  # 1: per-pair reciprocal-space cut (section "Integral screening")
    # > 0: compact/diffuse classification with this cutoff exponent (section
    # "Density classification: compact and diffuse"; the paper's default is omega^2/2)
    alpha_cut: float = 0.0
    dd_gpw: int = 0  # 1: the diffuse pairs through a real-space grid (GPW)

    @property
    def natm(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nshell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def nk(self) -> int:
        return int(self.kmesh[0] * self.kmesh[1] * self.kmesh[2])

    @property
    def nbf(self) -> int:
        return int(sum(ncart(int(l)) for l in self.shell_l))

    def shell_offsets(self) -> np.ndarray:
        off = np.zeros(self.nshell + 1, dtype=np.int64)
        for s, l in enumerate(self.shell_l):
            off[s + 1] = off[s] + ncart(int(l))
        return off

    def prim_offsets(self) -> np.ndarray:
        off = np.zeros(self.nshell + 1, dtype=np.int64)
        off[1:] = np.cumsum(self.shell_nprim)
        return off

    def kpoints_frac(self) -> np.ndarray:
        n1, n2, n3 = self.kmesh
        ks = []
        for m1 in range(n1):
            for m2 in range(n2):
                for m3 in range(n3):
                    ks.append((m1 / n1, m2 / n2, m3 / n3))
        return np.array(ks, dtype=np.float64)

    def with_(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# basis draws
# --------------------------------------------------------------------------

def draw_exponents(rng: np.random.Generator, counts: Sequence[int], lo: float, hi: float):
    """Per angular momentum l, counts[l] exponents exp(U(ln lo, ln hi)), sorted descending."""
    out = []
    for c in counts:
        e = np.exp(rng.uniform(math.log(lo), math.log(hi), size=int(c)))
        out.append(np.sort(e)[::-1].copy())
    return out


def build_problem(name, lattice, xyz, elements, element_exps, kmesh, omega, *,
                  eps_pair=1e-12, eps_G=1e-12, r_max=0.0, nelec=2.0, seed=0) -> Problem:
    """Uncontracted shells: one primitive per shell, coefficient 1.

    element_exps[el] is a list over l of exponent arrays; atoms of element el get
    one shell per exponent, ordered by l then by descending exponent.
    """
    sa, sl, sn, ex, co = [], [], [], [], []
    for ia, el in enumerate(elements):
        for l, arr in enumerate(element_exps[el]):
            for a in arr:
                sa.append(ia)
                sl.append(l)
                sn.append(1)
                ex.append(float(a))
                co.append(1.0)
    return Problem(
        name=name,
        lattice=np.asarray(lattice, dtype=np.float64).reshape(3, 3),
        xyz=np.asarray(xyz, dtype=np.float64).reshape(-1, 3),
        shell_atom=np.asarray(sa, dtype=np.int32),
        shell_l=np.asarray(sl, dtype=np.int32),
        shell_nprim=np.asarray(sn, dtype=np.int32),
        exps=np.asarray(ex, dtype=np.float64),
        coefs=np.asarray(co, dtype=np.float64),
        kmesh=tuple(int(k) for k in kmesh),
        omega=float(omega),
        eps_pair=float(eps_pair),
        eps_G=float(eps_G),
        r_max=float(r_max),
        nelec=float(nelec),
        seed=int(seed),
    )


# --------------------------------------------------------------------------
# the five workloads (cubic Gamma cell, diamond-like k-point cell, precision form
# of the first, rock-salt slab, monoclinic molecular crystal)
# --------------------------------------------------------------------------

def config_problem(i: int) -> Problem:
    if i in (1, 3):
        rng = np.random.default_rng(1)
        exps = {0: draw_exponents(rng, [4, 2], 0.1, 50.0)}
        a = 5.0
        return build_problem(
            "cubic2_gamma" if i == 1 else "cubic2_gamma_fp32",
            np.eye(3) * a, [[0, 0, 0], [2.5, 2.5, 2.5]], [0, 0], exps, (1, 1, 1), 0.5,
            r_max=15.0, nelec=8.0, seed=1)
    if i == 2:
        rng = np.random.default_rng(2)
        exps = {0: draw_exponents(rng, [10, 6, 3], 0.08, 2e4)}
        a = 6.74
        fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
        frac = np.vstack([fcc, fcc + 0.25])
        return build_problem("diamond8_k444", np.eye(3) * a, frac * a, [0] * 8, exps,
                             (4, 4, 4), 0.4, nelec=48.0, seed=2)
    if i == 4:
        rng = np.random.default_rng(4)
        exps = {0: draw_exponents(rng, [8, 5, 3, 1], 0.05, 5e4),
                1: draw_exponents(rng, [8, 5, 3, 1], 0.05, 5e4)}
        a = 7.96
        c = 1.5 * a + 20.0
        lat = np.array([[a, a, 0.0], [-a, a, 0.0], [0.0, 0.0, c]])
        ainv = np.linalg.inv(lat.T)
        xyz, els, seen = [], [], set()
        for k in range(4):
            for i1 in range(-4, 5):
                for j1 in range(-4, 5):
                    r = np.array([i1 * a / 2, j1 * a / 2, k * a / 2])
                    f = ainv @ r
                    key = tuple(np.round(np.mod(f[:2] + 1e-9, 1.0), 6)) + (k,)
                    if key in seen:
                        continue
                    seen.add(key)
                    fr = np.array([np.mod(f[0] + 1e-9, 1.0) - 1e-9, np.mod(f[1] + 1e-9, 1.0) - 1e-9, f[2]])
                    xyz.append(lat.T @ fr)
                    els.append(0 if (i1 + j1 + k) % 2 == 0 else 1)
        assert len(xyz) == 32, len(xyz)
        return build_problem("rocksalt_slab32_k661", lat, xyz, els, exps, (6, 6, 1), 0.4,
                             nelec=320.0, seed=4)
    if i == 5:
        rng = np.random.default_rng(5)
        exps = {0: draw_exponents(rng, [8, 4, 2], 0.1, 1e4),   # C
                1: draw_exponents(rng, [4, 2], 0.1, 1e4)}      # H
        a, b, c, beta = 14.0, 17.3, 7.3, 1.94
        lat = np.array([[a, 0, 0], [0, b, 0], [c * math.cos(beta), 0, c * math.sin(beta)]])
        centres = np.array([[0, 0, 0], [.5, .5, 0], [0, .5, .5], [.5, 0, .5]]) @ lat
        ang = np.arange(6) * math.pi / 3
        ring = np.stack([np.cos(ang), np.sin(ang), np.zeros(6)], axis=1)
        while True:
            xyz, els = [], []
            for cen in centres:
                R = _random_rotation(rng)
                for r in ring:
                    xyz.append(cen + R @ (2.64 * r))
                    els.append(0)
                for r in ring:
                    xyz.append(cen + R @ (4.69 * r))
                    els.append(1)
            xyz = np.array(xyz)
            if _min_image_distance(lat, xyz) >= 0.5:
                break
        return build_problem("benzene4_monoclinic_k333", lat, xyz, els, exps, (3, 3, 3), 0.5,
                             nelec=168.0, seed=5)
    raise ValueError(f"unknown config {i}")


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _min_image_distance(lat, xyz) -> float:
    best = np.inf
    n = len(xyz)
    for m in np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1])).T.reshape(-1, 3):
        L = m @ lat
        d = xyz[:, None, :] - xyz[None, :, :] - L
        r = np.linalg.norm(d, axis=2)
        if not m.any():
            r[np.arange(n), np.arange(n)] = np.inf
        best = min(best, float(r.min()))
    return best


# --------------------------------------------------------------------------
# overlap (used only to normalise the random densities)
# --------------------------------------------------------------------------

def _os_overlap_1d(la, lb, p, xpa, xpb, s00):
    """Obara-Saika 1D overlap table S[i][j], i<=la, j<=lb (vectorised over images)."""
    S = [[None] * (lb + 1) for _ in range(la + 1)]
    S[0][0] = s00
    inv2p = 0.5 / p
    for i in range(la + 1):
        for j in range(lb + 1):
            if i == 0 and j == 0:
                continue
            if i > 0:
                v = xpa * S[i - 1][j]
                if i > 1:
                    v = v + inv2p * (i - 1) * S[i - 2][j]
                if j > 0:
                    v = v + inv2p * j * S[i - 1][j - 1]
            else:
                v = xpb * S[i][j - 1]
                if j > 1:
                    v = v + inv2p * (j - 1) * S[i][j - 2]
            S[i][j] = v
    return S


def overlap_k(prob: Problem, eps: float = 1e-15) -> np.ndarray:
    """S_mu,nu(k) = sum_L e^{i k.L} S_mu,nu(L), complex [nk][nbf][nbf]."""
    lat = prob.lattice
    off = prob.shell_offsets()
    poff = prob.prim_offsets()
    kf = prob.kpoints_frac()
    nbf, nk = prob.nbf, prob.nk
    Sk = np.zeros((nk, nbf, nbf), dtype=np.complex128)
    B = 2 * math.pi * np.linalg.inv(lat)  # columns b_i, b_i . a_j = 2 pi delta_ij
    bn = np.linalg.norm(B, axis=0)
    for sa in range(prob.nshell):
        la = int(prob.shell_l[sa])
        A = prob.xyz[prob.shell_atom[sa]]
        ca = cart_components(la)
        for sb in range(prob.nshell):
            lb = int(prob.shell_l[sb])
            Bc = prob.xyz[prob.shell_atom[sb]]
            cb = cart_components(lb)
            block = np.zeros((nk, len(ca), len(cb)), dtype=np.complex128)
            for ia in range(poff[sa], poff[sa + 1]):
                aa, cA = prob.exps[ia], prob.coefs[ia]
                for ib in range(poff[sb], poff[sb + 1]):
                    ab, cB = prob.exps[ib], prob.coefs[ib]
                    p = aa + ab
                    mu = aa * ab / p
                    R = math.sqrt(-math.log(eps) / mu)
                    d = A - Bc
                    lo = np.floor((B.T @ d - bn * R) / (2 * math.pi)).astype(int) - 1
                    hi = np.ceil((B.T @ d + bn * R) / (2 * math.pi)).astype(int) + 1
                    ms = np.array(np.meshgrid(*[np.arange(lo[i], hi[i] + 1) for i in range(3)],
                                              indexing="ij")).reshape(3, -1).T
                    Ls = ms @ lat
                    Bp = Bc[None, :] + Ls
                    r2 = ((A[None, :] - Bp) ** 2).sum(1)
                    keep = mu * r2 <= -math.log(eps)
                    ms, Bp = ms[keep], Bp[keep]
                    if len(ms) == 0:
                        continue
                    P = (aa * A[None, :] + ab * Bp) / p
                    tabs = []
                    for x in range(3):
                        s00 = math.sqrt(math.pi / p) * np.exp(-mu * (A[x] - Bp[:, x]) ** 2)
                        tabs.append(_os_overlap_1d(la, lb, p, P[:, x] - A[x], P[:, x] - Bp[:, x], s00))
                    pref = cA * cB * gto_norm(la, aa) * gto_norm(lb, ab)
                    ph = np.exp(2j * math.pi * (kf @ ms.T))  # [nk][nimg]
                    for i, (ax, ay, az) in enumerate(ca):
                        for j, (bx, by, bz) in enumerate(cb):
                            sv = pref * tabs[0][ax][bx] * tabs[1][ay][by] * tabs[2][az][bz]
                            block[:, i, j] += ph @ sv
            Sk[:, off[sa]:off[sa + 1], off[sb]:off[sb + 1]] += block
    return Sk


# --------------------------------------------------------------------------
# densities
# --------------------------------------------------------------------------

def _minus_k_index(kmesh):
    n1, n2, n3 = kmesh
    idx = {}
    for m1 in range(n1):
        for m2 in range(n2):
            for m3 in range(n3):
                k = (m1 * n2 + m2) * n3 + m3
                mk = (((-m1) % n1) * n2 + (-m2) % n2) * n3 + (-m3) % n3
                idx[k] = mk
    return idx


def density_rank(prob: Problem) -> int:
    return prob.nbf if prob.nbf <= 512 else int(max(64, round(prob.nelec)))


def make_density(prob: Problem, seed: int, Sk: Optional[np.ndarray] = None,
                 rank: Optional[int] = None) -> np.ndarray:
    """Random Hermitian PSD D(k) = X_k X_k^H with time-reversal symmetry
    D(-k) = conj D(k) (real X at k = -k), scaled to sum_k w_k Tr(D(k) S(k)) = nelec.
    Returns complex128 [nk][nbf][nbf]."""
    rng = np.random.default_rng(seed)
    nbf, nk = prob.nbf, prob.nk
    r = density_rank(prob) if rank is None else rank
    mk = _minus_k_index(prob.kmesh)
    D = np.zeros((nk, nbf, nbf), dtype=np.complex128)
    for k in range(nk):
        if mk[k] < k:
            continue
        if mk[k] == k:
            X = rng.standard_normal((nbf, r))
            D[k] = X @ X.T
        else:
            X = rng.standard_normal((nbf, r)) + 1j * rng.standard_normal((nbf, r))
            D[k] = X @ X.conj().T
            D[mk[k]] = D[k].conj()
    if Sk is None:
        Sk = overlap_k(prob)
    ne = sum(np.sum(D[k] * Sk[k]).real for k in range(nk)) / nk
    D *= prob.nelec / ne
    return D


def make_densities(prob: Problem, ndm: int, base_seed: Optional[int] = None,
                   Sk: Optional[np.ndarray] = None) -> np.ndarray:
    """ndm densities with seeds 1000*seed + i, complex128 [ndm][nk][nbf][nbf]."""
    if Sk is None:
        Sk = overlap_k(prob)
    b = 1000 * prob.seed if base_seed is None else base_seed
    return np.stack([make_density(prob, b + i, Sk) for i in range(ndm)])


# --------------------------------------------------------------------------
# small systems for pins and parity cases
# --------------------------------------------------------------------------

def small_problem(kind: str = "sp", seed: int = 11, kmesh=(1, 1, 1), omega: float = 0.5,
                  lattice=None, lmax: int = 1, natm: int = 2, lo: float = 0.15, hi: float = 8.0,
                  r_max: float = 0.0, eps_pair: float = 1e-12, eps_G: float = 1e-12,
                  nper: int = 1) -> Problem:
    """A few-atom cell with nper shells per l <= lmax (one element), seeded positions."""
    rng = np.random.default_rng(seed)
    if lattice is None:
        lattice = np.array([[4.2, 0.0, 0.0], [0.3, 4.6, 0.0], [-0.4, 0.5, 3.9]])
    lattice = np.asarray(lattice, dtype=np.float64)
    exps = {0: draw_exponents(rng, [nper] * (lmax + 1), lo, hi)}
    frac = rng.uniform(0, 1, size=(natm, 3))
    xyz = frac @ lattice
    return build_problem(f"small_{kind}", lattice, xyz, [0] * natm, exps, kmesh, omega,
                         eps_pair=eps_pair, eps_G=eps_G, r_max=r_max,
                         nelec=2.0 * natm, seed=seed)



def diffuse_problem(seed: int = 7, a: float = 8.0, natm: int = 4, kmesh=(2, 2, 2), omega: float = 0.5) -> Problem:
    """A cell with diffuse shells for the compact/diffuse classification: natm
    atoms at seeded positions in a slightly skewed cell of side ~a Bohr, per atom
    s, p, d shells with one compact exponent each (2.2, 1.3, 0.9) and one just
    below alpha_cut = omega^2/2 (0.11, 0.115, 0.12 at omega = 0.5), so CC, CD and
    DD pairs of every class up to (2, 2) occur; alpha_cut is set."""
    rng = np.random.default_rng(seed)
    lat = np.array([[a, 0.0, 0.0], [0.05 * a, 1.04 * a, 0.0], [-0.07 * a, 0.08 * a, 0.95 * a]])
    xyz = rng.uniform(0, 1, size=(natm, 3)) @ lat
    ex = {0: [np.array([2.2, 0.11]), np.array([1.3, 0.115]), np.array([0.9, 0.12])]}
    prob = build_problem(f"diffuse{natm}_spd_a{a:g}", lat, xyz, [0] * natm, ex, kmesh, omega,
                         nelec=2.0 * natm, seed=seed)
    return prob.with_(alpha_cut=omega ** 2 / 2)


def make_densities_torch(prob: Problem, ndm: int, base_seed: int, Sk: np.ndarray, device="cuda", which=None):
    """Random Hermitian PSD D(k) with torch: the time-reversal-symmetric
    construction of make_density (D(k) = X_k X_k^H, D(-k) = conj D(k), real X at
    k = -k), each scaled to sum_k w_k Tr(D(k) S(k)) = nelec.  X ~ N(0,1) is drawn
    on the CPU from a torch generator seeded base_seed + i, so the densities are
    the same on any machine; the products run on `device` (a GPU for the large
    batches, "cpu" to rebuild a few of them for reference values).  which: the
    density indices to build (default range(ndm)).  Returns a complex128 tensor
    [len(which)][nk][nbf][nbf] on `device`."""
    import torch
    nbf, nk = prob.nbf, prob.nk
    r = density_rank(prob)
    mk = _minus_k_index(prob.kmesh)
    which = list(range(ndm)) if which is None else list(which)
    D = torch.empty((len(which), nk, nbf, nbf), dtype=torch.complex128, device=device)
    S = torch.from_numpy(np.ascontiguousarray(Sk)).to(device)
    for j, i in enumerate(which):
        g = torch.Generator(device="cpu")
        g.manual_seed(int(base_seed) + int(i))
        for k in range(nk):
            if mk[k] < k:
                continue
            if mk[k] == k:
                X = torch.randn((nbf, r), generator=g, dtype=torch.float64).to(device)
                D[j, k] = (X @ X.T.contiguous()).to(torch.complex128)
            else:
                Xr = torch.randn((nbf, r), generator=g, dtype=torch.float64)
                Xi = torch.randn((nbf, r), generator=g, dtype=torch.float64)
                X = torch.complex(Xr, Xi).to(device)
                D[j, k] = X @ X.conj().T.contiguous()
                D[j, mk[k]] = D[j, k].conj()
        ne = float((D[j] * S).real.sum()) / nk
        D[j] *= prob.nelec / ne
    del S
    return D
