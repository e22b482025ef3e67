"""GPU tests of the host drivers and the autograd Function over libtmm."""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _tmm():
    from paper_1410_0204_amd import tmm
    return tmm


def _obs(inp, seed=21):
    o = oracle.Oracle(inp)
    snaps = o.snapshots(synth.hidden_params(inp.model, seed=seed), inp.initial_state())
    return snaps * (1 + 0.05 * synth.obs_noise(snaps.shape, seed=seed + 1))


def test_autograd_function_gradients(tiny_ndop):
    import torch
    from paper_1410_0204_amd.autograd import year_misfit
    tmm = _tmm()
    inp = tiny_ndop
    obs = _obs(inp)
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1, adjoint_nbatch_max=1, ckpt_every=240)
    u = torch.tensor(synth.nominal(inp.model)[None, :], dtype=torch.float64, requires_grad=True)
    y0 = torch.as_tensor(inp.initial_state()).cuda().requires_grad_(True)
    J = year_misfit(u, y0, t, torch.as_tensor(obs).cuda())
    (3.0 * J.sum()).backward()
    eJ, eG, eY = oracle.Oracle(inp).year_adjoint(u.detach().numpy(), inp.initial_state(), obs)
    assert J.item() == pytest.approx(eJ[0], rel=1e-12)
    assert np.allclose(u.grad.numpy(), 3.0 * eG, rtol=1e-10, atol=0)
    g = y0.grad.cpu().numpy()
    assert np.abs(g - 3.0 * eY).max() <= 1e-10 * np.abs(3.0 * eY).max()


def test_newton_krylov_on_gpu(tiny_ndop):
    from paper_1410_0204_amd import drivers
    tmm = _tmm()
    inp = tiny_ndop
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1)
    u = synth.nominal(inp.model)
    y, hist = drivers.newton_krylov(t, u, inp.initial_state(), tol=1e-8, jvp="tangent", max_newton=12)
    phi, _ = oracle.Oracle(inp).year(u, y)
    assert np.linalg.norm(y - phi) <= 2e-8          # the oracle's year map agrees to its own rounding
    assert hist["fnorm"][-1] <= 1e-8


def test_spinup_residuals_match_oracle(small_ndop):
    from paper_1410_0204_amd import drivers
    tmm = _tmm()
    inp = small_ndop
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1)
    u = synth.nominal(inp.model)
    y, r = drivers.spinup(t, u, inp.initial_state(), years=3)
    ey, er = oracle.Oracle(inp).year(u, inp.initial_state(), 3)
    assert np.abs(y - ey).max() <= 1e-12 * np.abs(ey).max()
    assert np.allclose(r, er[:, 0], rtol=1e-9)


def test_ensemble_driver(small_ndop):
    from paper_1410_0204_amd import drivers
    tmm = _tmm()
    inp = small_ndop
    U = synth.latin_hypercube(synth.MODEL_NDOP, 20, seed=31)
    L = synth.spinup_lengths(20, seed=32, lo=1, hi=3)
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=20)
    y0 = inp.initial_state(20)
    out, resid = drivers.ensemble(t, U, L, y0)
    o = oracle.Oracle(inp)
    for m in (0, 7, 19):
        exp, er = o.year(U[m], y0[:, 2 * m:2 * m + 2], int(L[m]))
        assert np.abs(out[:, 2 * m:2 * m + 2] - exp).max() <= 1e-12 * np.abs(exp).max(), m
        assert np.allclose(resid[:L[m], m], er[:, 0], rtol=1e-9)


def test_autotuner_picks_a_validated_configuration(small_ndop, tmp_path):
    from paper_1410_0204_amd import autotune
    tmm = _tmm()
    inp = small_ndop
    for nb in (1, 20):
        U = synth.latin_hypercube(synth.MODEL_NDOP, nb, seed=50 + nb)
        t = tmm.TMM(inp.desc_arrays(), nbatch_max=nb)
        res = autotune.tune(t, U, inp.initial_state(nb), years=1)
        assert res["best"]["ok"] and len(res["candidates"]) >= 2
        path = str(tmp_path / "tuned.json")
        autotune.save(res, path)
        assert autotune.load(t, nb, path)["options"] == res["best"]["options"]
        # the tuned handle still reproduces the oracle
        t.set_params(U)
        got, _ = t.year(t.state(inp.initial_state(nb)))
        exp, _ = oracle.Oracle(inp).year(U, inp.initial_state(nb))
        assert np.abs(got.cpu().numpy() - exp).max() <= 1e-12 * np.abs(exp).max()


def test_trust_region_newton_on_gpu(tiny_ndop):
    from paper_1410_0204_amd import drivers
    tmm = _tmm()
    inp = tiny_ndop
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1)
    u = synth.nominal(inp.model)
    y, hist = drivers.newton_krylov(t, u, inp.initial_state(), tol=1e-8, jvp="tangent", max_newton=20,
                                    globalization="trust_region", delta0=1e-3)
    phi, _ = oracle.Oracle(inp).year(u, y)
    assert np.linalg.norm(y - phi) <= 2e-8
    assert hist["fnorm"][-1] <= 1e-8 and hist["newton"][0]["tau"] < 1.0


def test_preconditioned_newton_on_gpu(tiny_ndop):
    from paper_1410_0204_amd import drivers
    tmm = _tmm()
    inp = tiny_ndop
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1)
    u = synth.nominal(inp.model)
    y, hist = drivers.newton_krylov(t, u, inp.initial_state(), tol=1e-8, jvp="tangent", max_newton=20,
                                    preconditioner="transport")
    phi, _ = oracle.Oracle(inp).year(u, y)
    assert np.linalg.norm(y - phi) <= 2e-8
    V = inp.grid.volumes()
    assert (V @ y.sum(1)) == pytest.approx(V @ inp.initial_state().sum(1), rel=1e-10)
