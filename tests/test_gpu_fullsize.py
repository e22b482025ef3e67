"""GPU parity at full sizes, in the launch configurations bench.py times.

* global 128x64x15 (52749 points): the checkpointed adjoint of one model year
  (persistent kernels, checkpoints every 240 steps) against the oracle's
  full-trajectory reverse mode;
* ensemble 256x128x23 (500000 points, 64 members, W = 128): steps of the
  member-parallel kernel against the oracle's step, all outputs compared;
* 1.0-degree stand-in 360x180x23 (760000 points): a month of steps of the
  launch-per-step path against the oracle, and phosphorus conservation over
  one model year (a property that holds at any size).
"""

import numpy as np
import pytest

import oracle
import synth
from tolerances import ADJOINT, MISFIT, STEP, columnwise, componentwise, pointwise

pytestmark = pytest.mark.gpu


def test_global_adjoint_against_oracle():
    import torch
    from paper_1410_0204_amd import tmm
    inp = synth.global_2p8()
    o = oracle.Oracle(inp)
    y0 = inp.initial_state()
    print("[gpu] oracle snapshots and reverse mode on the global grid (~30 s)", flush=True)
    snaps = o.snapshots(synth.hidden_params(inp.model, seed=21), y0)
    obs = snaps * (1 + 0.05 * synth.obs_noise(snaps.shape, seed=22))
    u = synth.nominal(inp.model)
    eJ, eG, eY = o.year_adjoint(u, y0, obs)
    # checkpoints every 240 steps, and the whole year stored (no recomputation)
    for ckpt in (240, inp.nstep):
        print(f"[gpu] adjoint, ckpt_every={ckpt}", flush=True)
        t = tmm.TMM(inp.desc_arrays(), nbatch_max=1, adjoint_nbatch_max=1, ckpt_every=ckpt)
        assert t.query(tmm.TMM_Q_PERSISTENT) == 1
        t.set_params(u)
        J, G, dy0 = t.year_adjoint(t.state(y0), torch.as_tensor(obs).cuda())
        assert componentwise(J, eJ, f"global ckpt {ckpt} J") <= MISFIT, ckpt
        assert componentwise(G, eG, f"global ckpt {ckpt} dJ/du") <= ADJOINT, ckpt
        assert columnwise(dy0.cpu().numpy(), eY, 2, f"global ckpt {ckpt} dJ/dy0") <= ADJOINT, ckpt
        t.close()


def test_ensemble_steps_against_oracle():
    from paper_1410_0204_amd import tmm
    inp = synth.ensemble_1p4()
    nm = 64
    U = synth.latin_hypercube(synth.MODEL_NDOP, nm, seed=17)
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=nm)
    t.set_params(U)
    o = oracle.Oracle(inp)
    rng = np.random.default_rng(5)
    y = inp.initial_state(nm) * rng.uniform(0.8, 1.2, size=(inp.n, 2 * nm))
    yd = t.state(y)
    for j in (0, 1439):
        print(f"[gpu] ensemble step {j} on the oracle (~10 s)", flush=True)
        got = t.step(j, yd).cpu().numpy()
        exp = o.step(U, j, y)
        assert pointwise(got, exp, 2, f"ensemble step {j}") <= STEP, j
        # the tiled member kernel (bands of 2 latitude rows, 4 or 8 columns per workgroup): bit for bit
        t.set_option(tmm.TMM_OPT_MEMBER_BAND_ROWS, 2)
        for tile in (4, 8):
            print(f"[gpu] ensemble step {j}, tiled member kernel with {tile} columns", flush=True)
            t.set_option(tmm.TMM_OPT_MEMBER_TILE, tile)
            assert np.array_equal(t.step(j, yd).cpu().numpy(), got), (j, tile)
        t.set_option(tmm.TMM_OPT_MEMBER_TILE, 0)
        t.set_option(tmm.TMM_OPT_MEMBER_BAND_ROWS, 0)


def test_one_degree_month_and_conservation():
    """1.0-degree stand-in (360x180x23, 760000 points): 240 consecutive steps (one month, launch-per-step
    path) against the oracle, then one GPU model year conserves volume-weighted phosphorus."""
    from paper_1410_0204_amd import tmm
    inp = synth.one_degree()
    u = synth.nominal(inp.model)
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1)
    t.set_params(u)
    o = oracle.Oracle(inp)
    rng = np.random.default_rng(9)
    y = inp.initial_state() * rng.uniform(0.8, 1.2, size=(inp.n, 2))
    yd = t.state(y)
    print("[gpu] 240 steps on the 1-degree grid against the oracle (~20 s)", flush=True)
    for j in range(1320, 1560):
        yd = t.step(j, yd)
        y = o.step(u, j, y)
    assert pointwise(yd.cpu().numpy(), y, 2, "one degree, 240 steps") <= STEP
    y0 = inp.initial_state()
    y1, _ = t.year(t.state(y0))
    V = inp.grid.volumes()
    m0 = V @ y0.sum(1)
    m1 = V @ y1.cpu().numpy().sum(1)
    assert abs(m1 - m0) <= 1e-12 * m0
