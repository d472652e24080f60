"""E_J in real space on the device, 1/2 sum over (a, b, L) of D_ab(L) J_ab(L)
(section "Long-range contributions": the energy as the contraction of the
real-space blocks), against E_J of the same build (the G-space sum) and the
oracle, through the C ABI.

The two forms are the same quadratic form evaluated in a different order, so
they agree to rounding on every path: FP64 (with and without per-pair cuts), the
compact/diffuse classification by either DD route, the FP32-MFMA form, and graph
replay.  The bar is 1e-12 relative (a sum of ~1e5..1e6 terms of mixed sign).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_16460_amd import synth

from test_gpu_cd import cd_problem, gpw_problem
from test_gpu_parity import case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL = 1e-12


def pw():
    from paper_2509_16460_amd import pwdf
    return pwdf


CASES = {
    "spd_k123": lambda: case("spd_k123")[0],
    "spdf_k311_3atoms": lambda: case("spdf_k311_3atoms")[0],
    "contracted_k212_cut": lambda: case("contracted_k212")[0].with_(pair_gcut=1),
    "cd_spd_k211-aft": lambda: cd_problem(kmesh=(2, 1, 1), lmax=2, seed=61),
    "cd_spd_k211-gpw": lambda: gpw_problem(kmesh=(2, 1, 1), lmax=2, seed=64),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_real_space_energy_equals_g_space(name, prec):
    prob = CASES[name]()
    D = np.stack([synth.make_density(prob, 120 + i) for i in range(2)])
    ref = O.build_j(prob, D[0], want_J=False)
    ctx = pw().LongRangeJ(prob, precision=prec, max_ndm=2)
    Dt = torch.from_numpy(D).cuda()
    _, E = ctx.build_j(Dt)
    ER = ctx.energy_real().cpu().numpy()
    E = E.cpu().numpy()
    for i in range(2):
        print(f"{name} prec {prec} density {i}: E_G={E[i]:.15f} E_R={ER[i]:.15f} "
              f"dE={abs(E[i] - ER[i]):.2e} rel={abs(E[i] - ER[i]) / abs(E[i]):.2e}")
        assert abs(E[i] - ER[i]) <= REL * max(1.0, abs(E[i]))
    assert abs(ER[0] - ref["E_G"]) <= (1e-10 if prec == 0 else 1e-7)
    # graph replay leaves the same blocks behind
    _, Eg = ctx.build_j(Dt, graph=True)
    ERg = ctx.energy_real().cpu().numpy()
    assert np.array_equal(ERg, ER) and np.array_equal(Eg.cpu().numpy(), E)
    # the first density of the batch alone
    ER1 = ctx.energy_real(ndm=1).cpu().numpy()
    assert ER1[0] == ER[0]


def test_real_space_energy_needs_the_blocks_of_a_build():
    prob = case("sp_k221")[0]
    D = torch.from_numpy(synth.make_density(prob, 130)[None]).cuda()
    ctx = pw().LongRangeJ(prob, precision=0, max_ndm=2)
    with pytest.raises(pw().PwdfError, match="holds the D"):
        ctx.energy_real(ndm=1)
    ctx.build_j(D)
    ctx.energy_real()
    with pytest.raises(pw().PwdfError, match="holds the D"):
        ctx.energy_real(ndm=2)
    ctx.get_rhoG(D)
    with pytest.raises(pw().PwdfError, match="holds the D"):
        ctx.energy_real(ndm=1)
    ctx.build_j(D)
    ctx.build_j(D, noalloc=True)
    with pytest.raises(pw().PwdfError, match="holds the D"):
        ctx.energy_real(ndm=1)
