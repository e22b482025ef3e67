"""tmm_year_noalloc (the entry point for callers that cannot allocate) against tmm_year.

Both run the same kernels; the non-allocating one keeps its buffers in the
library's fixed device array, which every call on the device shares and
which keeps the previous call's contents.  Two calls in a row, the second on
a smaller input (another handle, fewer points and members), must each equal
tmm_year's result; a request too large for the array is refused before
anything runs.
"""

import numpy as np
import pytest

import oracle
import synth
from tolerances import YEAR, pointwise

pytestmark = pytest.mark.gpu


def _tmm():
    from paper_1410_0204_amd import tmm
    return tmm


def test_noalloc_matches_year_twice_then_smaller():
    tmm = _tmm()
    # first call: 3 members on the 32x16x8 grid (tile kernel), two years into a separate output
    big = synth.small_ndop()
    U = synth.latin_hypercube(synth.MODEL_NDOP, 3, seed=61)
    ta = tmm.TMM(big.desc_arrays(), nbatch_max=3)
    ta.set_params(U)
    rng = np.random.default_rng(62)
    y0 = big.initial_state(3) * rng.uniform(0.8, 1.2, size=(big.n, 6))
    print("[gpu] noalloc call 1: small grid, 3 members, 2 years", flush=True)
    out = ta.state()
    got, r = ta.year_noalloc(ta.state(y0), out, nyears=2)
    exp, re = ta.year(ta.state(y0), nyears=2)
    assert bool((got == exp).all())                     # same kernels, same order: bit for bit
    assert np.array_equal(r, re)
    assert pointwise(got.cpu().numpy(), oracle.Oracle(big).year(U, y0, 2)[0], 2, "noalloc call 1") <= YEAR

    # second call: one member on the 16x8x4 grid, in place (y1 = y0), one year
    small = synth.tiny(model=synth.MODEL_NDOP)
    tb = tmm.TMM(small.desc_arrays(), nbatch_max=1)
    u = synth.nominal(synth.MODEL_NDOP)
    tb.set_params(u)
    s0 = small.initial_state()
    print("[gpu] noalloc call 2: tiny grid, 1 member, in place", flush=True)
    yd = tb.state(s0)
    got2, r2 = tb.year_noalloc(yd, yd, nyears=1)
    tb.set_option(tmm.TMM_OPT_PERSISTENT, 0)
    exp2, re2 = tb.year(tb.state(s0), nyears=1)
    assert bool((got2 == exp2).all())
    assert np.array_equal(r2, re2)
    tb.set_option(tmm.TMM_OPT_PERSISTENT, 1)
    exp3, re3 = tb.year(tb.state(s0), nyears=1)          # the single-launch kernel: same to rounding
    assert pointwise(got2.cpu().numpy(), exp3.cpu().numpy(), 2, "noalloc call 2 vs single launch") <= YEAR
    assert r2[0, 0] == pytest.approx(re3[0, 0], rel=1e-9)


def test_noalloc_member_kernel_and_no_sync_path():
    tmm = _tmm()
    inp = synth.small_ndop()
    U = synth.latin_hypercube(synth.MODEL_NDOP, 20, seed=63)
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=20)
    t.set_params(U)
    y0 = t.state(inp.initial_state(20))
    print("[gpu] noalloc: 20 members (member kernel), no residuals, no check", flush=True)
    t.set_option(tmm.TMM_OPT_CHECK_FINITE, 0)
    out = t.state()
    got, r = t.year_noalloc(y0, out, nyears=1, residuals=False)
    assert r is None
    import torch
    torch.cuda.synchronize()
    exp, _ = t.year(y0, nyears=1, residuals=False)
    assert bool((got == exp).all())


def test_noalloc_refuses_what_does_not_fit():
    tmm = _tmm()
    inp = synth.small_ndop()
    nb = 400                                           # 2 n W = 4.3 million doubles > 32 MiB
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=nb)
    t.set_params(synth.latin_hypercube(synth.MODEL_NDOP, nb, seed=64))
    y0 = t.state(inp.initial_state(nb))
    out = t.state()
    out.fill_(7.0)
    with pytest.raises(tmm.TmmError) as err:
        t.year_noalloc(y0, out, nyears=1)
    assert err.value.status == tmm.TMM_ETOOBIG
    assert bool((out == 7.0).all())                   # nothing ran
