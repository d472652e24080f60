"""Launch runtime of the HIP path (needs an MI355X).

* fork/join over the context's internal streams is deterministic: two eager
  calls, and an eager call with profiling on (everything on one stream), give
  bit-identical J(k) and E_J;
* pwdf_build_j_graph: the captured graph, replayed several times with other
  eager work and new D(k) contents between replays, reproduces the eager result
  of each density bit for bit (same kernels, same shapes, no memset nodes);
* pwdf_autotune: the tuned context still meets the FP64 bar against the oracle,
  writes a cache entry, and a second context applies the cached shapes without
  timing (same segment length, bit-identical results to the first tuned one);
* E_J of a J build (summed by an extra block of the J(k) launch) and of the
  gradient path (its own energy launch) come from the same partials in the same
  order: bit-identical, eager and graph-replayed, for a batch of two densities.
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


def problem():
    return synth.small_problem(kind="runtime", seed=61, kmesh=(2, 1, 2), lmax=3, natm=2, lo=0.3, hi=18.0)


def dev(D):
    return torch.from_numpy(np.ascontiguousarray(D[None] if D.ndim == 3 else D)).cuda()


def test_fork_join_deterministic():
    p = problem()
    D = synth.make_density(p, 611)
    ctx = pw().LongRangeJ(p, max_ndm=1)
    J1, E1 = ctx.build_j(dev(D))
    J2, E2 = ctx.build_j(dev(D))
    ctx.profile_enable(True)
    J3, E3 = ctx.build_j(dev(D))
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    torch.cuda.synchronize()
    assert torch.equal(J1, J2) and torch.equal(E1, E2)
    assert torch.equal(J1, J3) and torch.equal(E1, E3)
    assert any(k.startswith("rho_") for k in prof) and "phase_j" in prof


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_mfma"])
def test_graph_replay_matches_eager(prec):
    p = problem()
    ndm = 2
    ctx = pw().LongRangeJ(p, precision=prec, max_ndm=ndm)
    other = pw().LongRangeJ(p, precision=prec, max_ndm=1)
    dens = [np.stack([synth.make_density(p, 620 + 2 * r), synth.make_density(p, 621 + 2 * r)]) for r in range(4)]
    Dbuf = dev(dens[0])
    Jg = torch.empty_like(Dbuf)
    Eg = torch.empty(ndm, dtype=torch.float64, device="cuda")
    for r, D in enumerate(dens):
        Dbuf.copy_(dev(D))
        ctx.build_j(Dbuf, Jg, Eg, graph=True)
        torch.cuda.synchronize()
        Jr, Er = Jg.clone(), Eg.clone()
        # eager work of the program between replays: another context and torch ops
        Jo, _ = other.build_j(dev(D[0]))
        (Jo.abs() * 2).sum().item()
        # eager reference on the same context, separate output buffers
        Je, Ee = ctx.build_j(dev(D))
        torch.cuda.synchronize()
        print(f"prec={prec} replay {r}: max|dJ|={float((Jr - Je).abs().max()):.1e}", flush=True)
        assert torch.equal(Jr, Je), f"replay {r}: J differs from the eager call"
        assert torch.equal(Er, Ee), f"replay {r}: E_J differs from the eager call"
        if prec == 0:
            assert torch.equal(Jo[0], Je[0])
        else:
            # max_ndm = 1 gives the FP32-MFMA form other column layouts and chunks:
            # equal up to that form's rounding
            assert float((Jo[0] - Je[0]).abs().max()) <= 1e-9 * float(Je[0].abs().max())


def test_graph_recaptures_on_new_buffers():
    p = problem()
    ctx = pw().LongRangeJ(p, max_ndm=1)
    D = synth.make_density(p, 630)
    Ja, Ea = ctx.build_j(dev(D), graph=True)
    Jb, Eb = ctx.build_j(dev(D), graph=True)  # new buffers: captured again
    Je, Ee = ctx.build_j(dev(D))
    torch.cuda.synchronize()
    assert torch.equal(Ja, Je) and torch.equal(Jb, Je) and torch.equal(Ea, Ee) and torch.equal(Eb, Ee)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_mfma"])
def test_autotune_parity_and_cache(prec, tmp_path):
    p = problem()
    D = synth.make_density(p, 640)
    ref = O.build_j(p, D, want_J=True, want_rho=False)
    ctx = pw().LongRangeJ(p, precision=prec, max_ndm=1)
    J0, E0 = ctx.build_j(dev(D))
    cache = str(tmp_path / "tune.txt")
    ctx.autotune(1, cache)
    seg = ctx.stats()["seg_len"]
    J1, E1 = ctx.build_j(dev(D))
    torch.cuda.synchronize()
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and int(lines[0].split()[1]) == int(seg)
    e_tol, j_tol = (1e-10, 1e-11) if prec == 0 else (1e-6, 1e-6)
    dE = abs(float(E1.cpu()[0]) - ref["E_G"])
    dJ = float(np.max(np.abs(J1.cpu().numpy()[0] - ref["J"])))
    print(f"prec={prec} seg={seg} dE={dE:.2e} dJ={dJ:.2e}", flush=True)
    assert dE <= e_tol and dJ <= j_tol
    if prec == 0:
        assert float((J1 - J0).abs().max()) <= 1e-13
    # a second context takes the cached shapes without timing
    ctx2 = pw().LongRangeJ(p, precision=prec, max_ndm=1)
    ctx2.autotune(1, cache)
    assert ctx2.stats()["seg_len"] == seg
    J2, E2 = ctx2.build_j(dev(D))
    torch.cuda.synchronize()
    assert torch.equal(J1, J2) and torch.equal(E1, E2)
    assert len(open(cache).read().strip().splitlines()) == 1


def test_autotune_full_diamond_cell():
    """Diamond 8-atom cell, 4x4x4 mesh: tuned FP64 path vs untuned (summation order only)."""
    p = synth.config_problem(2)
    D = synth.make_density(p, 2000)
    ctx = pw().LongRangeJ(p, max_ndm=1)
    J0, E0 = ctx.build_j(dev(D))
    ctx.autotune(1, None)
    J1, E1 = ctx.build_j(dev(D))
    Jg, Eg = ctx.build_j(dev(D), graph=True)
    torch.cuda.synchronize()
    dJ = float((J1 - J0).abs().max())
    dE = abs(float(E1.cpu()[0]) - float(E0.cpu()[0]))
    print(f"diamond tuned seg={ctx.stats()['seg_len']} dE={dE:.2e} dJ={dJ:.2e}", flush=True)
    assert dE <= 1e-11 and dJ <= 1e-12
    assert torch.equal(Jg, J1) and torch.equal(Eg, E1)


# the FP32-MFMA pair-G kernels walk a compact list of G points; its slot layout
# uses 8-point segments only
@pytest.mark.parametrize("prec,segs", [(0, (4, 5, 8, 16)), (1, (8,))], ids=["fp64", "fp32_mfma"])
def test_every_segment_length_matches_oracle(prec, segs, tmp_path):
    """Each segment length the kernels are built for, forced through a tune-cache
    entry (applied without timing), against the oracle; a length the kernels are
    not built for is rejected."""
    p = synth.small_problem(kind="segs", seed=71, kmesh=(2, 2, 1), lmax=2, natm=2, lo=0.2, hi=12.0)
    D = synth.make_density(p, 710)
    ref = O.build_j(p, D, want_J=True, want_rho=False)
    probe = pw().LongRangeJ(p, precision=prec, max_ndm=1)
    cache = tmp_path / "tune.txt"
    probe.autotune(1, str(cache))
    key = cache.read_text().split()[0]
    ones = " ".join(["1"] * 16)
    e_tol, j_tol = (1e-10, 1e-11) if prec == 0 else (1e-6, 1e-6)
    for seg in segs:
        cache.write_text(f"{key} {seg} {ones}\n")
        ctx = pw().LongRangeJ(p, precision=prec, max_ndm=1)
        ctx.autotune(1, str(cache))
        assert ctx.stats()["seg_len"] == seg
        J, E = ctx.build_j(dev(D))
        torch.cuda.synchronize()
        dE = abs(float(E.cpu()[0]) - ref["E_G"])
        dJ = float(np.max(np.abs(J.cpu().numpy()[0] - ref["J"])))
        print(f"prec={prec} seg={seg} nseg={ctx.stats()['nseg']} dE={dE:.2e} dJ={dJ:.2e}", flush=True)
        assert dE <= e_tol and dJ <= j_tol
    cache.write_text(f"{key} {7 if prec == 0 else 4} {ones}\n")
    ctx = pw().LongRangeJ(p, precision=prec, max_ndm=1)
    with pytest.raises(pw().PwdfError) as ei:
        ctx.autotune(1, str(cache))
    assert ei.value.status == -1


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_mfma"])
def test_fork_setting_from_cache(prec, tmp_path):
    """The launches of a pass overlapping on internal streams (fork 1) or in
    sequence on the caller's stream (fork 0), and for the FP32-MFMA form in the
    order of given launch times, set through a tune-cache entry: bit-identical
    J(k) and E_J, eager and replayed as a graph."""
    p = problem()
    D = dev(synth.make_density(p, 650))
    probe = pw().LongRangeJ(p, precision=prec, max_ndm=1)
    cache = tmp_path / "tune.txt"
    probe.autotune(1, str(cache))
    assert probe.stats()["fork"] in (0, 1)
    key = cache.read_text().split()[0]
    ones = " ".join(["1"] * 16)
    out = {}
    # FP32-MFMA form: also the per-class launches ordered by (made-up) launch times,
    # longest first onto the least-loaded stream ("1 1 <costs>")
    costs = " ".join(f"{(7 * i) % 11 + 0.5:g}" for i in range(32))
    variants = [("1", 1), ("0", 0)] + ([(f"1 1 {costs}", 1)] if prec == 1 else [])
    for tail, fk in variants:
        cache.write_text(f"{key} 8 {ones} {tail}\n")
        ctx = pw().LongRangeJ(p, precision=prec, max_ndm=1)
        ctx.autotune(1, str(cache))
        assert ctx.stats()["fork"] == fk
        Je, Ee = ctx.build_j(D)
        Jg, Eg = ctx.build_j(D, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(Je, Jg) and torch.equal(Ee, Eg)
        out[tail] = (Je, Ee)
    for tail, _ in variants[1:]:
        assert torch.equal(out[tail][0], out["1"][0]) and torch.equal(out[tail][1], out["1"][1])


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_mfma"])
def test_energy_same_bits_on_every_path(prec):
    p = problem()
    D = np.stack([synth.make_density(p, 631), synth.make_density(p, 632)])
    ctx = pw().LongRangeJ(p, precision=prec, max_ndm=2)
    Dt = dev(D)
    _, E_eager = ctx.build_j(Dt)
    J = torch.empty_like(Dt)
    E_graph = torch.empty(2, dtype=torch.float64, device="cuda")
    for _ in range(2):
        ctx.build_j(Dt, J, E_graph, graph=True)
    _, E_grad = ctx.grad(Dt)
    torch.cuda.synchronize()
    a, b, c = (x.cpu().numpy() for x in (E_eager, E_graph, E_grad))
    print(f"E_J eager {a} graph {b} gradient path {c}", flush=True)
    assert np.array_equal(a, b) and np.array_equal(a, c)
    for i in range(2):
        ref = O.build_j(p, D[i], want_J=False, want_rho=False)
        assert abs(a[i] - ref["E_G"]) <= (1e-10 if prec == 0 else 1e-7)

