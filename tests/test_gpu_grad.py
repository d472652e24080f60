"""Nuclear gradient dE_J/dR at fixed D(k), pair list and G set (needs an MI355X).

* against the oracle's analytic gradient (FP64): <= 1e-10 relative to max |g|;
* translation invariance: sum_A dE/dR_A = 0;
* central finite differences of the GPU FP64 energy, delta = 1e-4 Bohr, with the
  same pair count at the displaced geometries (truncation ~ delta^2 E''' / 6);
* the autograd Function: xyz.grad = pwdf_grad, and the D(k) gradient
  w_k conj J(k) matches a finite difference along a Hermitian direction;
* the molecular-crystal workload (48 atoms, 3x3x3 k-mesh) at full size: E_J,
  the gradient of all atoms and sampled J(k) against the oracle (stored
  values), sum rule, finite differences for two atoms in FP64 and FP32-MFMA.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_16460_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def pw():
    from paper_2509_16460_amd import pwdf
    return pwdf


def grad_gpu(prob, D, prec=0):
    ctx = pw().LongRangeJ(prob, precision=prec, max_ndm=1)
    g, E = ctx.grad(torch.from_numpy(D[None]).cuda())
    torch.cuda.synchronize()
    return g.cpu().numpy()[0], float(E.cpu()[0]), ctx


def energy_gpu(prob, D, prec=0):
    ctx = pw().LongRangeJ(prob, precision=prec, max_ndm=1)
    _, E = ctx.build_j(torch.from_numpy(D[None]).cuda())
    torch.cuda.synchronize()
    return float(E.cpu()[0]), ctx.stats()["npairs"]


CASES = {
    "sp_k211": dict(kind="g1", seed=81, kmesh=(2, 1, 1), lmax=1, natm=3, lo=0.3, hi=12.0),
    "spd_gamma": dict(kind="g2", seed=82, lmax=2, natm=2, lo=0.3, hi=15.0),
    "spdf_k121": dict(kind="g3", seed=83, kmesh=(1, 2, 1), lmax=3, natm=2, lo=0.4, hi=10.0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_grad_vs_oracle(name):
    p = synth.small_problem(**CASES[name])
    D = synth.make_density(p, 91)
    ref = O.build_j(p, D, want_J=False, want_rho=False, want_grad=True)
    g, E, _ = grad_gpu(p, D)
    scale = np.max(np.abs(ref["grad"]))
    print(f"{name}: max|g|={scale:.3e} max|dg|={np.max(np.abs(g - ref['grad'])):.2e}", flush=True)
    assert abs(E - ref["E_G"]) <= 1e-10
    assert np.max(np.abs(g - ref["grad"])) <= 1e-10 * max(1.0, scale)
    assert np.max(np.abs(g.sum(0))) <= 1e-11 * max(1.0, scale)


def fd_check(prob, D, atoms, delta=1e-4, prec=0):
    g, E0, ctx = grad_gpu(prob, D, prec)
    n0 = ctx.stats()["npairs"]
    worst = 0.0
    for a in atoms:
        for c in range(3):
            xp = prob.xyz.copy()
            xm = prob.xyz.copy()
            xp[a, c] += delta
            xm[a, c] -= delta
            Ep, npp = energy_gpu(prob.with_(xyz=xp), D, prec)
            Em, npm = energy_gpu(prob.with_(xyz=xm), D, prec)
            assert npp == n0 and npm == n0, "pair list changed under the displacement"
            fd = (Ep - Em) / (2 * delta)
            worst = max(worst, abs(fd - g[a, c]))
    return worst, np.max(np.abs(g)), g


def test_grad_finite_differences():
    p = synth.small_problem(**CASES["spd_gamma"])
    D = synth.make_density(p, 92)
    worst, scale, _ = fd_check(p, D, atoms=[0, 1])
    print(f"FD: worst |fd - g| = {worst:.2e} (max|g| {scale:.2e})", flush=True)
    assert worst <= 1e-7 * max(1.0, scale)


def test_grad_fp32_form():
    p = synth.small_problem(**CASES["sp_k211"])
    D = synth.make_density(p, 93)
    g64, _, _ = grad_gpu(p, D, 0)
    g32, _, _ = grad_gpu(p, D, pw().PWDF_FP32_MFMA)
    rel = np.max(np.abs(g32 - g64)) / np.max(np.abs(g64))
    print(f"FP32 gradient rel err {rel:.2e}", flush=True)
    assert rel <= 1e-8


def test_autograd_function():
    p = synth.small_problem(**CASES["sp_k211"])
    D = synth.make_density(p, 94)
    plan = pw().LongRangeJ(p, max_ndm=1)
    Dt = torch.from_numpy(D[None]).cuda().requires_grad_(True)
    xyz = torch.from_numpy(p.xyz.copy()).requires_grad_(True)
    E = pw().long_range_energy(Dt, xyz, plan)
    E.sum().backward()
    g, _ = plan.grad(torch.from_numpy(D[None]).cuda())
    assert torch.allclose(xyz.grad, g.cpu()[0], rtol=0, atol=1e-14)
    # directional derivative along a Hermitian, time-reversal-symmetric direction
    X = synth.make_density(p, 95)
    h = 1e-3
    Jp, Ep = plan.build_j(torch.from_numpy((D + h * X)[None]).cuda())
    Jm, Em = plan.build_j(torch.from_numpy((D - h * X)[None]).cuda())
    fd = (float(Ep.cpu()[0]) - float(Em.cpu()[0])) / (2 * h)
    an = float(torch.sum(Dt.grad.conj().cpu() * torch.from_numpy(X[None])).real)
    assert abs(fd - an) <= 1e-9 * max(1.0, abs(an))


@pytest.fixture(scope="module")
def crystal():
    f = np.load(os.path.join(GOLDEN, "molecular_crystal.npz"))
    p = synth.config_problem(5)
    D = synth.make_density(p, int(f["density_seed"]))
    return p, D, f


def test_molecular_crystal_vs_oracle(crystal):
    """48-atom monoclinic cell, 3x3x3 mesh, FP64: E_J, the analytic gradient of all
    48 atoms and J(k) at 12k sampled support elements against the oracle (stored
    values, tests/golden/molecular_crystal.npz)."""
    p, D, f = crystal
    g, E, ctx = grad_gpu(p, D)
    J, EJ = ctx.build_j(torch.from_numpy(D[None]).cuda())
    torch.cuda.synchronize()
    idx = f["idx"]
    Js = J.cpu().numpy()[0][idx[:, 0], idx[:, 1], idx[:, 2]]
    scale = float(np.max(np.abs(f["grad"])))
    dE = abs(E - float(f["E_G"]))
    dEb = abs(float(EJ.cpu()[0]) - float(f["E_G"]))
    dg = float(np.max(np.abs(g - f["grad"])))
    dJ = float(np.max(np.abs(Js - f["J"])))
    print(f"molecular crystal FP64 vs oracle: E_J={E:.12f} dE={dE:.2e} (build {dEb:.2e}) max|dg|={dg:.2e} "
          f"(max|g| {scale:.2e}) max|dJ|={dJ:.2e} (max|J| {float(f['maxJ']):.2e})", flush=True)
    assert dE <= 1e-10 and dEb <= 1e-10
    assert dg <= 1e-10 * max(1.0, scale)
    assert dJ <= 1e-11 * max(1.0, float(f["maxJ"]))
    assert np.max(np.abs(g.sum(0))) <= 1e-10 * max(1.0, scale)


def test_molecular_crystal_finite_differences(crystal):
    """Central differences (delta = 1e-4 Bohr) for two atoms, FP64 and FP32-MFMA.
    The FP32 form's energies carry rounding of the FP32 tiles; most of it is the
    same at the displaced geometries (same pairs, same G set), the rest enters the
    difference quotient divided by 2 delta: its bar is 4 |E32 - E64| / delta on
    top of the FD truncation, with E32 - E64 measured at the base geometry."""
    p, D, _ = crystal
    worst, scale, g = fd_check(p, D, atoms=[0, 17])
    print(f"molecular crystal FP64: max|g|={scale:.3e} worst FD err {worst:.2e}", flush=True)
    assert worst <= 1e-7 * max(1.0, scale)
    E64, _ = energy_gpu(p, D, 0)
    E32, _ = energy_gpu(p, D, pw().PWDF_FP32_MFMA)
    worst32, scale32, g32 = fd_check(p, D, atoms=[0, 17], prec=pw().PWDF_FP32_MFMA)
    bar = 4 * abs(E32 - E64) / 1e-4 + 1e-7 * max(1.0, scale)
    rel = np.max(np.abs(g32 - g)) / scale
    print(f"molecular crystal FP32-MFMA: |E32-E64|={abs(E32 - E64):.2e} worst FD err {worst32:.2e} "
          f"(bar {bar:.2e}); gradient vs FP64 rel {rel:.2e}", flush=True)
    assert worst32 <= bar
    assert rel <= 1e-6
