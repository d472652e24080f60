#!/usr/bin/env python
"""Writes the oracle reference values of the two largest workloads (CPU only).

The FP64 oracle takes minutes on these cells (and longer with the gradient), so
the GPU tests compare against values stored here instead of running it.  Every
value is computed by oracle/ alone from the seeded inputs of
paper_2509_16460_amd/synth.py; nothing comes from the HIP library.

  molecular_crystal.npz  monoclinic cell, 4 C6H6-shaped molecules (48 atoms),
                         3x3x3 mesh, omega 0.5, density seed 5000:
                         E_J by its three routes, the analytic gradient of all
                         48 atoms, and J(k) at a seeded sample of support
                         elements covering every shell-pair class.
  slab.npz               rock-salt slab, 32 atoms, 6x6x1 mesh, omega 0.4,
                         densities 0 and 11 of the 16-density batch
                         (synth.make_densities_torch, base seed 4000): E_J and
                         J(k) at a seeded sample of support elements.

    python tests/golden/make_fixtures.py [crystal] [slab]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2509_16460_amd import synth  # noqa: E402

NSAMPLE = 12000


def support_sample(prob, nsample, seed):
    """(k, mu, nu) of J(k) elements on the pair support: the same number drawn
    from every shell-pair class (la, lb) present, the rest uniformly."""
    P = O.pairs(prob)
    off = prob.shell_offsets()
    rng = np.random.default_rng(seed)
    by_cls = {}
    for sa, sb in sorted({(int(r[0]), int(r[1])) for r in P}):
        cl = (int(prob.shell_l[sa]), int(prob.shell_l[sb]))
        for mu in range(off[sa], off[sa + 1]):
            for nu in range(off[sb], off[sb + 1]):
                by_cls.setdefault(cl, []).append((mu, nu))
    per = nsample // len(by_cls)
    picks = []
    for cl in sorted(by_cls):
        els = np.array(by_cls[cl], dtype=np.int64)
        sel = rng.choice(len(els), size=min(per, len(els)), replace=False)
        picks.append(els[sel])
    els = np.concatenate(picks)
    ks = rng.integers(0, prob.nk, size=len(els))
    return np.stack([ks, els[:, 0], els[:, 1]], axis=1).astype(np.int32)


def crystal():
    prob = synth.config_problem(5)
    D = synth.make_density(prob, 5000)
    t = time.time()
    r = O.build_j(prob, D, want_rho=False, want_grad=True)
    print(f"crystal oracle: {time.time() - t:.0f} s  E_J={r['E_G']:.12f}", flush=True)
    idx = support_sample(prob, NSAMPLE, 5001)
    J = r["J"][idx[:, 0], idx[:, 1], idx[:, 2]]
    np.savez_compressed(os.path.join(HERE, "molecular_crystal.npz"), density_seed=5000, E_G=r["E_G"],
                        E_real=r["E_real"], E_k=r["E_k"], grad=r["grad"], idx=idx, J=J,
                        maxJ=np.max(np.abs(r["J"])))


def slab():
    prob = synth.config_problem(4)
    Sk = synth.overlap_k(prob)
    which = [0, 11]
    Dt = synth.make_densities_torch(prob, 16, 1000 * prob.seed, Sk, device="cpu", which=which)
    out = {"which": np.array(which), "base_seed": 1000 * prob.seed}
    for j, i in enumerate(which):
        t = time.time()
        r = O.build_j(prob, Dt[j].numpy(), want_rho=False)
        print(f"slab density {i} oracle: {time.time() - t:.0f} s  E_J={r['E_G']:.10f}", flush=True)
        idx = support_sample(prob, NSAMPLE, 4100 + i)
        out[f"E_G_{i}"] = r["E_G"]
        out[f"idx_{i}"] = idx
        out[f"J_{i}"] = r["J"][idx[:, 0], idx[:, 1], idx[:, 2]]
        out[f"maxJ_{i}"] = np.max(np.abs(r["J"]))
    np.savez_compressed(os.path.join(HERE, "slab.npz"), **out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["crystal", "slab"]
    if "slab" in which:
        slab()
    if "crystal" in which:
        crystal()
