"""GPU tests of the host drivers and the autograd Function over libtmm."""

import numpy as np
import pytest

import oracle
import synth
from tolerances import ADJOINT, YEAR, columnwise, pointwise

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
    assert columnwise(y0.grad.cpu().numpy(), 3.0 * eY, 2, "autograd dJ/dy0") <= ADJOINT


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
    assert pointwise(y, ey, 2, "spin-up, three years") <= YEAR
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
        assert pointwise(out[:, 2 * m:2 * m + 2], exp, 2, f"ensemble driver member {m}") <= YEAR, m
        assert np.allclose(resid[:L[m], m], er[:, 0], rtol=1e-9)


@pytest.mark.parametrize("nb", [1, 20])
def test_autotuner_candidates_match_the_oracle(small_ndop, tmp_path, nb):
    """Every candidate the autotuner tries (domain sizes of the single-launch kernel, tile sizes of the
    tile kernel, wave counts and column orders of the member kernel, the tiled member kernel) gives the
    oracle's model year; the tuned table round-trips and the drivers apply it."""
    from paper_1410_0204_amd import autotune
    tmm = _tmm()
    inp = small_ndop
    U = synth.latin_hypercube(synth.MODEL_NDOP, nb, seed=50 + nb)
    y0 = inp.initial_state(nb)
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=nb)
    t.set_params(U)
    exp, _ = oracle.Oracle(inp).year(U, y0)
    cands = autotune.candidates(t, nb)
    assert len(cands) >= (13 if nb == 1 else 19)
    for cand in cands:
        autotune.apply(t, autotune.DEFAULTS)
        autotune.apply(t, cand)
        got, _ = t.year(t.state(y0), residuals=False)
        assert pointwise(got.cpu().numpy(), exp, 2, f"nb {nb} {autotune.describe(cand)}") <= YEAR, cand
    res = autotune.tune(t, U, y0, years=1)
    assert res["best"]["ok"] and len(res["candidates"]) == len(cands)
    path = str(tmp_path / "tuned.json")
    autotune.save(res, path)
    t2 = tmm.TMM(inp.desc_arrays(), nbatch_max=nb)
    rec = autotune.apply_tuned(t2, nb, path)
    assert rec is not None and rec["options"] == res["best"]["options"]
    t2.set_params(U)
    got, _ = t2.year(t2.state(y0), residuals=False)
    assert pointwise(got.cpu().numpy(), exp, 2, f"nb {nb} tuned") <= YEAR


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


def test_newton_fixed_point_is_the_spinup_limit_on_gpu(small_ndop):
    """The periodic solution of section 4 found by Newton-Krylov (section 6) is where spin-up goes:
    on the 32x16x8 grid spin-up is run until its residual is 1e-10 (it contracts by about 2.6 % a
    year, so several hundred years) and must then agree with the Newton solution at the same total
    mass, to the spin-up's own residual divided by its contraction gap."""
    from paper_1410_0204_amd import drivers
    tmm = _tmm()
    inp = small_ndop
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1)
    u = synth.nominal(inp.model)
    y0 = inp.initial_state()
    ystar, hist = drivers.newton_krylov(t, u, y0, tol=1e-10, jvp="tangent", max_newton=20)
    assert hist["fnorm"][-1] <= 1e-10
    print(f"[gpu] Newton: {len(hist['newton'])} steps, {hist['years']} year maps", flush=True)
    y, r, mass = drivers.spinup(t, u, y0, years=4000, tol=1e-10, return_mass=True)
    rho = (r[-1] / r[-51]) ** (1 / 50)
    print(f"[gpu] spin-up: {len(r)} years to residual {r[-1]:.3e}, rate {rho:.4f}", flush=True)
    assert r[-1] <= 1e-10
    V = inp.grid.volumes()
    assert V @ ystar.sum(1) == pytest.approx(V @ y0.sum(1), rel=1e-11)
    assert abs(mass[-1].sum() / mass[0].sum() - 1.0) <= 1e-11
    err = np.linalg.norm(y - ystar)
    print(f"[gpu] |spin-up limit - Newton| = {err:.3e}", flush=True)
    assert err <= 2.0 * r[-1] / (1.0 - rho) + 1e-9
