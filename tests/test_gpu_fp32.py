"""FP32-MFMA form vs the FP64 oracle / FP64 path (needs an MI355X).

Targets of the precision form: |E_J - E_J(oracle)| <= 1e-7 Eh and
max |J(k) - J(k)(oracle)| <= 1e-8, on the cubic Gamma cell (2 atoms, 4s2p per
atom) and on small cells with every class up to (3,3) (also within 2e-8
relative of the FP64 path).  Batched calls must give, density by density, the
same result as single-density FP32 calls up to that form's rounding (1e-8).
The head of the G set (the G whose Coulomb weight is within 2^-20 of the
largest; pwdf_set_fp32_head) is contracted with FP64 tiles; a head that covers
the whole G set takes every pair-G product in FP64 and meets the FP64 bars.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_16460_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def pw():
    from paper_2509_16460_amd import pwdf
    return pwdf


def run(prob, D, prec, max_ndm=None):
    ndm = D.shape[0]
    ctx = pw().LongRangeJ(prob, precision=prec, max_ndm=max_ndm or ndm)
    J, E = ctx.build_j(torch.from_numpy(np.ascontiguousarray(D)).cuda())
    torch.cuda.synchronize()
    return J.cpu().numpy(), E.cpu().numpy()


def test_cubic_gamma_fp32_targets():
    p = synth.config_problem(3)
    D = synth.make_density(p, 1000)
    ref = O.build_j(p, D, want_rho=False)
    J, E = run(p, D[None], pw().PWDF_FP32_MFMA)
    dE = abs(E[0] - ref["E_G"])
    dJ = np.max(np.abs(J[0] - ref["J"]))
    print(f"cubic Gamma FP32-MFMA: E_J={E[0]:.12f} dE={dE:.3e} max|dJ|={dJ:.3e} (max|J|={np.max(np.abs(ref['J'])):.3e})",
          flush=True)
    assert dE <= 1e-7
    assert dJ <= 1e-8


@pytest.mark.parametrize("name,lmax,kmesh,natm", [("sp", 1, (2, 1, 1), 2), ("spd", 2, (1, 2, 2), 2),
                                                  ("spdf", 3, (1, 1, 1), 2)])
def test_fp32_vs_fp64_classes(name, lmax, kmesh, natm):
    p = synth.small_problem(kind=name, seed=60 + lmax, kmesh=kmesh, lmax=lmax, natm=natm, lo=0.25, hi=30.0)
    D = synth.make_density(p, 61)[None]
    ref = O.build_j(p, D[0], want_rho=False)
    J64, E64 = run(p, D, pw().PWDF_FP64)
    J32, E32 = run(p, D, pw().PWDF_FP32_MFMA)
    relE = abs(E32[0] - E64[0]) / abs(E64[0])
    relJ = np.max(np.abs(J32 - J64)) / np.max(np.abs(J64))
    dE = abs(E32[0] - ref["E_G"])
    dJ = np.max(np.abs(J32[0] - ref["J"]))
    print(f"{name}: relE={relE:.2e} relJ={relJ:.2e} vs oracle: dE={dE:.2e} max|dJ|={dJ:.2e}", flush=True)
    assert relE <= 2e-8 and relJ <= 2e-8
    assert dE <= 1e-7 and dJ <= 1e-8


def test_head_weight_moves_work_into_fp64():
    """pwdf_set_fp32_head: a smaller weight puts more G in the FP64 head; a head
    that covers the whole G set meets the FP64 bars against the oracle."""
    p = synth.small_problem(kind="hw", seed=66, kmesh=(2, 1, 1), lmax=2, natm=2, lo=0.25, hi=30.0)
    D = synth.make_density(p, 67)
    ref = O.build_j(p, D, want_rho=False)
    ctx = pw().LongRangeJ(p, precision=pw().PWDF_FP32_MFMA, max_ndm=1)
    n_default = ctx.stats()["nG_head"]
    ctx.set_fp32_head(2.0 ** -7)
    n7 = ctx.stats()["nG_head"]
    ctx.set_fp32_head(1e-300)
    st = ctx.stats()
    assert 0 < n7 <= n_default <= st["nG_head"] == st["nG"] // 2
    assert abs(st["pairG_head"] - st["pairG_evals"]) <= 1e-9 * st["pairG_evals"]
    J, E = ctx.build_j(torch.from_numpy(D[None]).cuda())
    torch.cuda.synchronize()
    dE = abs(float(E.cpu()[0]) - ref["E_G"])
    dJ = float(np.max(np.abs(J.cpu().numpy()[0] - ref["J"])))
    print(f"all-FP64 head: dE={dE:.2e} max|dJ|={dJ:.2e} (heads {n7} / {n_default} / {st['nG_head']})", flush=True)
    assert dE <= 1e-10 and dJ <= 1e-11
    with pytest.raises(pw().PwdfError, match="PWDF_EINVAL"):
        ctx.set_fp32_head(0.0)


@pytest.mark.parametrize("ndm", [3, 16])
def test_fp32_batched_equals_single(ndm):
    p = synth.small_problem(kind="b", seed=70, kmesh=(2, 1, 1), lmax=2, natm=2, lo=0.25, hi=20.0)
    D = np.stack([synth.make_density(p, 700 + i) for i in range(ndm)])
    Jb, Eb = run(p, D, pw().PWDF_FP32_MFMA)
    J64, E64 = run(p, D, pw().PWDF_FP64)
    for i in (0, ndm - 1):
        Js, Es = run(p, D[i:i + 1], pw().PWDF_FP32_MFMA)
        assert abs(Eb[i] - Es[0]) <= 1e-8 * abs(Es[0])
        assert np.max(np.abs(Jb[i] - Js[0])) <= 1e-8 * np.max(np.abs(Js[0]))
    relE = np.max(np.abs(Eb - E64) / np.abs(E64))
    relJ = np.max(np.abs(Jb - J64)) / np.max(np.abs(J64))
    print(f"batched ndm={ndm}: relE={relE:.2e} relJ={relJ:.2e}", flush=True)
    assert relE <= 2e-8 and relJ <= 2e-8
