"""GPU parity for the PO4-DOP-PHY model (section 2.2.2): three tracers, eleven parameters.

Every path of libtmm with W = 3 per member against the oracle: the tile step
kernel, the single-launch year kernel and the launch-per-step year, the
tangent (both paths), the persistent and tile adjoints, batches through the
tile kernel, and one model year on the global grid.  Tolerances as for the
other models (states point by point, signed fields per tracer column,
gradients per component, as in ``tolerances.py``): one step 1e-14, one model
year 1e-12, tangent 1e-11, adjoint 1e-10.
"""

import numpy as np
import pytest

import oracle
import synth
from tolerances import ADJOINT, MISFIT, STEP, TANGENT, YEAR, columnwise, componentwise, pointwise

pytestmark = pytest.mark.gpu

PHY = synth.MODEL_NDOPPHY


def _tmm():
    from paper_1410_0204_amd import tmm
    return tmm


@pytest.fixture(scope="module")
def inputs():
    return {"tiny": synth.tiny(model=PHY), "small": synth.small_ndop(model=PHY)}


def _make(inp, nbatch_max=1, adjoint=0, ckpt=240):
    print(f"[gpu] create {inp.name} model={inp.model} nbatch_max={nbatch_max} adjoint={adjoint}", flush=True)
    return _tmm().TMM(inp.desc_arrays(), nbatch_max=nbatch_max, adjoint_nbatch_max=adjoint, ckpt_every=ckpt)


def _state(inp, nb=1, seed=1):
    rng = np.random.default_rng(seed)
    return inp.initial_state(nb) * rng.uniform(0.5, 1.5, size=(inp.n, 3 * nb))


@pytest.mark.parametrize("name", ["tiny", "small"])
def test_phy_step_parity(inputs, name):
    inp = inputs[name]
    t = _make(inp)
    o = oracle.Oracle(inp)
    u = synth.nominal(PHY)
    t.set_params(u)
    y = _state(inp)
    for j in (0, 119, 1439, 2879):
        got = t.step(j, t.state(y)).cpu().numpy()
        exp = o.step(u, j, y)
        assert pointwise(got, exp, 3, f"PHY {name} step {j}") <= STEP, j


@pytest.mark.parametrize("persistent", [1, 0])
@pytest.mark.parametrize("name", ["tiny", "small"])
def test_phy_year_parity(inputs, name, persistent):
    tmm = _tmm()
    inp = inputs[name]
    t = _make(inp)
    t.set_option(tmm.TMM_OPT_PERSISTENT, persistent)
    o = oracle.Oracle(inp)
    u = synth.nominal(PHY)
    t.set_params(u)
    y0 = inp.initial_state()
    got, r = t.year(t.state(y0), nyears=2)
    exp, re = o.year(u, y0, 2)
    assert pointwise(got.cpu().numpy(), exp, 3, f"PHY {name} two years, path {persistent}") <= YEAR
    assert np.allclose(r, re, rtol=1e-9, atol=0)


def test_phy_batch_through_tile_kernel(inputs):
    inp = inputs["small"]
    U = synth.latin_hypercube(PHY, 3, seed=31)
    t = _make(inp, nbatch_max=3)
    t.set_params(U)
    y0 = _state(inp, 3, seed=32)
    got, _ = t.year(t.state(y0))
    exp, _ = oracle.Oracle(inp).year(U, y0)
    assert pointwise(got.cpu().numpy(), exp, 3, "PHY batch of 3") <= YEAR


@pytest.mark.parametrize("persistent", [1, 0])
def test_phy_tangent(inputs, persistent):
    tmm = _tmm()
    inp = inputs["small"]
    t = _make(inp)
    t.set_option(tmm.TMM_OPT_PERSISTENT, persistent)
    o = oracle.Oracle(inp)
    u = synth.nominal(PHY)
    t.set_params(u)
    rng = np.random.default_rng(13)
    y = _state(inp, seed=14)
    v = rng.standard_normal(y.shape) * y
    phi, jv = t.year_jvp(t.state(y), t.state(v), mode=tmm.TMM_JVP_TANGENT)
    ephi, ejv = o.year_tangent(u, y, v)
    assert pointwise(phi.cpu().numpy(), ephi, 3) <= YEAR
    assert columnwise(jv.cpu().numpy(), ejv, 3, f"PHY tangent, path {persistent}") <= TANGENT


def _obs(inp, o, seed=21):
    snaps = o.snapshots(synth.hidden_params(PHY, seed=seed), inp.initial_state())
    return snaps * (1 + 0.05 * synth.obs_noise(snaps.shape, seed=seed + 1))


@pytest.mark.parametrize("persistent", [1, 0])
@pytest.mark.parametrize("name,ckpt", [("tiny", 240), ("small", 480)])
def test_phy_adjoint(inputs, name, ckpt, persistent):
    import torch
    tmm = _tmm()
    inp = inputs[name]
    o = oracle.Oracle(inp)
    obs = _obs(inp, o)
    u = synth.nominal(PHY)
    y0 = inp.initial_state()
    eJ, eG, eY = o.year_adjoint(u, y0, obs)
    t = _make(inp, adjoint=1, ckpt=ckpt)
    t.set_option(tmm.TMM_OPT_PERSISTENT, persistent)
    t.set_params(u)
    J, G, dy0 = t.year_adjoint(t.state(y0), torch.as_tensor(obs).cuda())
    assert componentwise(J, eJ, f"PHY {name} ckpt {ckpt} J") <= MISFIT
    assert componentwise(G, eG, f"PHY {name} ckpt {ckpt} dJ/du") <= ADJOINT
    assert columnwise(dy0.cpu().numpy(), eY, 3, f"PHY {name} ckpt {ckpt} dJ/dy0") <= ADJOINT


@pytest.mark.parametrize("ckpt", [240, 2880])
def test_phy_ensemble_adjoint(inputs, ckpt):
    import torch
    inp = inputs["tiny"]
    U = synth.latin_hypercube(PHY, 2, seed=3)
    o = oracle.Oracle(inp)
    obs1 = _obs(inp, o)
    obs = np.concatenate([obs1, obs1 * 1.02], axis=2)
    y0 = inp.initial_state(2)
    eJ, eG, eY = o.year_adjoint(U, y0, obs)
    t = _make(inp, nbatch_max=2, adjoint=2, ckpt=ckpt)
    t.set_params(U)
    J, G, dy0 = t.year_adjoint(t.state(y0), torch.as_tensor(obs).cuda())
    assert componentwise(J, eJ, f"PHY two members ckpt {ckpt} J") <= MISFIT
    assert componentwise(G, eG, f"PHY two members ckpt {ckpt} dJ/du") <= ADJOINT
    assert columnwise(dy0.cpu().numpy(), eY, 3, f"PHY two members ckpt {ckpt} dJ/dy0") <= ADJOINT


def test_phy_global_year():
    """Full size: one model year of the global grid with three tracers (single-launch kernel)."""
    tmm = _tmm()
    inp = synth.global_2p8(model=PHY)
    t = _make(inp)
    assert t.query(tmm.TMM_Q_PERSISTENT) == 1
    u = synth.nominal(PHY)
    t.set_params(u)
    y0 = inp.initial_state()
    got, _ = t.year(t.state(y0))
    print("[gpu] oracle year, global grid, PO4-DOP-PHY (~15 s)", flush=True)
    exp, _ = oracle.Oracle(inp).year(u, y0)
    assert pointwise(got.cpu().numpy(), exp, 3, "PHY global year") <= YEAR
