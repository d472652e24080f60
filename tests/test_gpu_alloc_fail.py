"""Device allocation failures, forced through the library's test hook
(pwdf_debug_fail_alloc): every setup that runs out of memory returns
PWDF_ENOMEM and releases what it had allocated, pwdf_create returns no context,
a context whose re-setup failed answers PWDF_ESTATE to device work, and
pwdf_destroy leaves no allocation behind.  Each allocation of a context's setup
is made to fail in turn, on a cell with DD pairs on the GPW route (every
optional workspace present) in both precision forms.
"""
import numpy as np
import pytest

from paper_2509_16460_amd import synth

from test_gpu_cd import gpw_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ENOMEM, ESTATE = -2, -6


def pw():
    from paper_2509_16460_amd import pwdf
    return pwdf


@pytest.fixture(autouse=True)
def no_injected_failures():
    yield
    pw().lib().pwdf_debug_fail_alloc(-1)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_failed_creation_releases_everything(prec):
    L = pw().lib()
    prob = gpw_problem(kmesh=(2, 1, 1), lmax=1, seed=67)
    base = L.pwdf_debug_live_allocs()
    ctx = pw().LongRangeJ(prob, precision=prec, max_ndm=2)
    n = L.pwdf_debug_live_allocs() - base
    ctx.close()
    assert n > 10 and L.pwdf_debug_live_allocs() == base
    for k in range(n):
        L.pwdf_debug_fail_alloc(k)
        with pytest.raises(pw().PwdfError) as ei:
            pw().LongRangeJ(prob, precision=prec, max_ndm=2)
        L.pwdf_debug_fail_alloc(-1)
        assert ei.value.status == ENOMEM, str(ei.value)
        assert L.pwdf_debug_live_allocs() == base, f"allocation {k} of {n} failed: leak"
    print(f"prec {prec}: {n} device allocations per setup, each failed in turn, none leaked")


def test_failed_resetup_leaves_the_context_unusable():
    L = pw().lib()
    prob = gpw_problem(kmesh=(2, 1, 1), lmax=1, seed=67)
    D = torch.from_numpy(synth.make_density(prob, 91)[None]).cuda()
    base = L.pwdf_debug_live_allocs()
    ctx = pw().LongRangeJ(prob, precision=1, max_ndm=1)
    J0, E0 = ctx.build_j(D)
    torch.cuda.synchronize()
    L.pwdf_debug_fail_alloc(5)
    with pytest.raises(pw().PwdfError) as ei:
        ctx.set_fp32_head(2.0 ** -16)
    L.pwdf_debug_fail_alloc(-1)
    assert ei.value.status == ENOMEM
    # the partial setup is released already; device work is refused
    assert L.pwdf_debug_live_allocs() == base
    for call in (lambda: ctx.build_j(D), lambda: ctx.build_j(D, graph=True), lambda: ctx.grad(D),
                 lambda: ctx.get_rhoG(D), lambda: ctx.energy_real(ndm=1), lambda: ctx.check_input(),
                 lambda: ctx.autotune(1)):
        with pytest.raises(pw().PwdfError) as ei:
            call()
        assert ei.value.status == ESTATE, str(ei.value)
    ctx.close()
    assert L.pwdf_debug_live_allocs() == base
    # a new context on the same device works and gives the same result
    ctx = pw().LongRangeJ(prob, precision=1, max_ndm=1)
    J1, E1 = ctx.build_j(D)
    torch.cuda.synchronize()
    assert torch.equal(J0, J1) and torch.equal(E0, E1)
    ctx.close()
    assert L.pwdf_debug_live_allocs() == base
