"""GPU parity on degenerate and extreme inputs, against the oracle.

* a grid of one wet point (one column of one layer, one workgroup, one domain);
* a grid whose columns are all no deeper than the euphotic zone (every export
  remineralised in a bottom layer);
* the shortest year the month interpolation allows (24 steps: two per month,
  the month pair changes every other step) and a single monthly matrix
  (nmat = 1, no interpolation, two steps a year);
* 24-layer columns (the persistent kernels with 32-entry column blocks and
  256-thread workgroups) and 64-layer columns (the deepest the library takes:
  launch-per-step kernels only);
* zero model years (the state comes back unchanged).
Each case runs steps, a year on every available path, the tangent and the
adjoint, to the usual tolerances.  With fewer steps per year the rates
(alpha, lambda'_2) are scaled by nstep/2880 so that dt times each rate is that
of the standard configuration; otherwise the explicit Euler production
overshoots, N goes negative and rounding differences grow without bound.
"""

import numpy as np
import pytest

import oracle
import synth
from tolerances import ADJOINT, MISFIT, STEP, TANGENT, YEAR, columnwise, componentwise, pointwise

pytestmark = pytest.mark.gpu

CASES = {
    "point": dict(nlon=1, nlat=1, nlayer=1, ncol=1, n=1, neuphotic=1),
    "shallow": dict(nlon=8, nlat=4, nlayer=2, ncol=20, n=33, neuphotic=2),
    "short_year": dict(nlon=8, nlat=4, nlayer=4, ncol=20, n=50, nstep=24),
    "one_matrix": dict(nlon=8, nlat=4, nlayer=4, ncol=20, n=50, nmat=1, nstep=2),
    "deep24": dict(nlon=32, nlat=16, nlayer=24, ncol=300, n=5000),
    "deep64": dict(nlon=8, nlat=8, nlayer=64, ncol=40, n=1800),
}
CKPT = {"short_year": 4, "one_matrix": 1}


def _tmm():
    from paper_1410_0204_amd import tmm
    return tmm


@pytest.fixture(scope="module")
def inputs():
    return {k: synth.custom(**kw) for k, kw in CASES.items()}


def _params(inp, u=None):
    u = synth.nominal(inp.model) if u is None else u.copy()
    u[0] *= inp.nstep / 2880.0
    u[4] *= inp.nstep / 2880.0
    return u


def _make(inp, name, adjoint=0):
    print(f"[gpu] create {name} n={inp.n} nlayer={inp.grid.nlayer} nstep={inp.nstep} nmat={inp.nmat}", flush=True)
    ckpt = CKPT.get(name, 240)
    return _tmm().TMM(inp.desc_arrays(), nbatch_max=1, adjoint_nbatch_max=adjoint, ckpt_every=ckpt)


@pytest.mark.parametrize("name", list(CASES))
def test_edge_steps_and_years(inputs, name):
    tmm = _tmm()
    inp = inputs[name]
    t = _make(inp, name)
    o = oracle.Oracle(inp)
    u = _params(inp)
    t.set_params(u)
    rng = np.random.default_rng(7)
    y = inp.initial_state() * rng.uniform(0.5, 1.5, size=(inp.n, inp.ntracer))
    for j in sorted({0, 1, inp.nstep // 2, inp.nstep - 1}):
        assert pointwise(t.step(j, t.state(y)).cpu().numpy(), o.step(u, j, y), inp.ntracer,
                         f"{name} step {j}") <= STEP, j
    exp, re = o.year(u, y, 2)
    paths = [1, 0] if t.query(tmm.TMM_Q_PERSISTENT) else [0]
    if name == "deep24":
        assert paths == [1, 0]        # the persistent kernels with 32-entry blocks are exercised
    if name == "deep64":
        assert paths == [0]
    for pers in paths:
        t.set_option(tmm.TMM_OPT_PERSISTENT, pers)
        got, r = t.year(t.state(y), nyears=2)
        assert pointwise(got.cpu().numpy(), exp, inp.ntracer, f"{name} two years, path {pers}") <= YEAR, pers
        # a residual near zero is rounding noise: compare it against the state's size
        assert np.abs(r - re).max() <= 1e-9 * np.abs(re).max() + 1e-12 * np.linalg.norm(exp), pers
    same, _ = t.year(t.state(y), nyears=0)
    assert np.array_equal(same.cpu().numpy(), y)


@pytest.mark.parametrize("name", list(CASES))
def test_edge_tangent_and_adjoint(inputs, name):
    import torch
    tmm = _tmm()
    inp = inputs[name]
    o = oracle.Oracle(inp)
    u = _params(inp)
    rng = np.random.default_rng(8)
    y = inp.initial_state() * rng.uniform(0.8, 1.2, size=(inp.n, inp.ntracer))
    v = rng.standard_normal(y.shape) * y
    _, ejv = o.year_tangent(u, y, v)
    snaps = o.snapshots(_params(inp, synth.hidden_params(inp.model, seed=21)), inp.initial_state())
    obs = snaps * (1 + 0.05 * synth.obs_noise(snaps.shape, seed=22))
    eJ, eG, eY = o.year_adjoint(u, inp.initial_state(), obs)
    t = _make(inp, name, adjoint=1)
    t.set_params(u)
    paths = [1, 0] if t.query(tmm.TMM_Q_PERSISTENT) else [0]
    for pers in paths:
        t.set_option(tmm.TMM_OPT_PERSISTENT, pers)
        _, jv = t.year_jvp(t.state(y), t.state(v), mode=tmm.TMM_JVP_TANGENT)
        assert columnwise(jv.cpu().numpy(), ejv, inp.ntracer, f"{name} tangent, path {pers}") <= TANGENT, pers
        J, G, dy0 = t.year_adjoint(t.state(inp.initial_state()), torch.as_tensor(obs).cuda())
        assert componentwise(J, eJ, f"{name} J, path {pers}") <= MISFIT, pers
        assert componentwise(G, eG, f"{name} dJ/du, path {pers}") <= ADJOINT, pers
        assert columnwise(dy0.cpu().numpy(), eY, inp.ntracer, f"{name} dJ/dy0, path {pers}") <= ADJOINT, pers


def test_wait_give_up_is_reported_and_the_handle_recovers():
    """A wait of the persistent kernel that gives up is reported, and leaves nothing behind.

    The failure is forced from the host: a spin limit of one poll makes any wait
    that needs a second poll give up (with many small domains some wait in a model
    year always does).  The kernel still ends normally; the call reports
    TMM_EDEVICE.  With the default limit restored, the next year on the same handle
    matches the oracle.
    """
    tmm = _tmm()
    inp = synth.small_ndop()
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1)
    t.set_option(tmm.TMM_OPT_DOMAIN_ROWS, 16)
    assert t.query(tmm.TMM_Q_PERSISTENT) == 1
    print(f"[gpu] forced give-up, {t.query(tmm.TMM_Q_DOMAINS)} domains", flush=True)
    u = synth.nominal(inp.model)
    t.set_params(u)
    y0 = inp.initial_state()
    t.set_option(tmm.TMM_OPT_SPIN_LIMIT, 1)
    with pytest.raises(tmm.TmmError) as err:
        t.year(t.state(y0), nyears=1)
    assert err.value.status == tmm.TMM_EDEVICE
    t.set_option(tmm.TMM_OPT_SPIN_LIMIT, 0)
    got, _ = t.year(t.state(y0), nyears=1)
    exp, _ = oracle.Oracle(inp).year(u, y0)
    assert pointwise(got.cpu().numpy(), exp, inp.ntracer, "after the give-up") <= YEAR


@pytest.mark.parametrize("persistent", [1, 0])
def test_nonfinite_year_is_reported(persistent):
    """A NaN in the initial state makes tmm_year return TMM_ENONFINITE (the per-year check of the
    state), once: the next finite year on the same handle is clean and matches the oracle.  With
    the check off the same call succeeds.  The kernels run to completion either way (a NaN is
    never the persistent kernel's empty-slot marker)."""
    tmm = _tmm()
    inp = synth.small_ndop()
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1)
    t.set_option(tmm.TMM_OPT_PERSISTENT, persistent)
    print(f"[gpu] NaN input, persistent={persistent}", flush=True)
    u = synth.nominal(inp.model)
    t.set_params(u)
    y0 = inp.initial_state()
    bad = y0.copy()
    bad[100, 1] = np.nan
    with pytest.raises(tmm.TmmError) as err:
        t.year(t.state(bad))
    assert err.value.status == tmm.TMM_ENONFINITE
    got, _ = t.year(t.state(y0))
    exp, _ = oracle.Oracle(inp).year(u, y0)
    assert pointwise(got.cpu().numpy(), exp, 2, f"after a NaN year, path {persistent}") <= YEAR
    t.set_option(tmm.TMM_OPT_CHECK_FINITE, 0)
    out, _ = t.year(t.state(bad))
    assert np.isnan(out.cpu().numpy()).any()


def test_exchange_probe():
    """The latency probe runs its bounded ping-pong, barrier and load chains to the end and reports
    positive, finite latencies (and where its workgroups ran)."""
    tmm = _tmm()
    inp = synth.tiny()
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1)
    p = t.probe_exchange(500)
    print(f"[gpu] probe: {p}", flush=True)
    for k in ("round_trip_same_xcd_us", "round_trip_cross_xcd_us", "barrier_us", "agent_load_us"):
        assert 0.0 < p[k] < 1000.0, k
    assert all(0 <= x < 16 for x in p["xcds"])


def test_member_kernel_rows_without_diagonal():
    """The member-parallel kernel takes a row's own DOP from the stencil slot that reads the row
    itself: the diagonal entry, or, in a row without one, a zero padding entry (the ELL table is
    widened when the longest row lacks its diagonal).  Rows of both kinds, 20 members, steps
    against the oracle."""
    import copy
    tmm = _tmm()
    inp = copy.deepcopy(synth.small_ndop())
    tm = inp.tm
    lens = np.diff(tm.ae_rowptr)
    col = tm.ae_colidx.copy()
    for i in (int(np.argmax(lens)), int(np.argmin(lens)), inp.n // 2):
        e0, e1 = tm.ae_rowptr[i], tm.ae_rowptr[i + 1]
        row = set(col[e0:e1].tolist())
        spare = next(c for c in range(inp.n) if c not in row)
        col[e0 + list(col[e0:e1]).index(i)] = spare       # the diagonal's value now acts on another row
    tm.ae_colidx = col
    nb = 20
    U = synth.latin_hypercube(synth.MODEL_NDOP, nb, seed=44)
    print(f"[gpu] member kernel, rows without diagonal, {nb} members", flush=True)
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=nb)
    t.set_option(tmm.TMM_OPT_MEMBER_KERNEL_MIN, 1)
    t.set_params(U)
    o = oracle.Oracle(inp)
    rng = np.random.default_rng(45)
    y = inp.initial_state(nb) * rng.uniform(0.7, 1.3, size=(inp.n, 2 * nb))
    for j in (0, 1439, 2879):
        got = t.step(j, t.state(y)).cpu().numpy()
        exp = o.step(U, j, y)
        assert pointwise(got, exp, 2, f"rows without diagonal, step {j}") <= STEP, j


@pytest.mark.parametrize("grid", ["few_latitudes", "many_latitudes"])
def test_persistent_insolation_table_and_its_fallback(grid):
    """The persistent forward kernel holds the year's insolation of its domain's latitude rows in
    LDS; a domain spanning more than 8 latitude rows (here: two columns per latitude row, one
    domain) loads it every step instead.  Both against the oracle, forward year and tangent."""
    tmm = _tmm()
    if grid == "few_latitudes":
        inp = synth.small_ndop()
    else:
        inp = synth.custom(nlon=2, nlat=40, nlayer=4, ncol=60, n=200, model=synth.MODEL_NDOP)
    print(f"[gpu] insolation table, {grid}: n={inp.n}", flush=True)
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1)
    assert t.query(tmm.TMM_Q_PERSISTENT) == 1
    assert t.query(tmm.TMM_Q_INSOLATION_LDS) == (1 if grid == "few_latitudes" else 0)
    o = oracle.Oracle(inp)
    u = synth.nominal(inp.model)
    t.set_params(u)
    rng = np.random.default_rng(46)
    y = inp.initial_state() * rng.uniform(0.8, 1.2, size=(inp.n, 2))
    got, _ = t.year(t.state(y))
    exp, _ = o.year(u, y)
    assert pointwise(got.cpu().numpy(), exp, 2, f"insolation {grid}, one year") <= YEAR
    v = rng.standard_normal(y.shape) * y
    phi, jv = t.year_jvp(t.state(y), t.state(v), mode=tmm.TMM_JVP_TANGENT)
    ephi, ejv = o.year_tangent(u, y, v)
    assert columnwise(jv.cpu().numpy(), ejv, 2, f"insolation {grid}, tangent") <= TANGENT


def test_persistent_wave_aligned_and_packed_columns():
    """The persistent forward kernels place every water column within one wavefront (one workgroup
    barrier per step, the LDS state alternating between two buffers) or, with the option off, pack
    the columns (three barriers per step).  Same arithmetic per row: both layouts give the same
    year and tangent bit for bit, and both match the oracle."""
    tmm = _tmm()
    inp = synth.small_ndop()
    print(f"[gpu] wave-aligned and packed columns: n={inp.n}", flush=True)
    t = tmm.TMM(inp.desc_arrays(), nbatch_max=1)
    o = oracle.Oracle(inp)
    u = synth.nominal(inp.model)
    t.set_params(u)
    rng = np.random.default_rng(47)
    y = inp.initial_state() * rng.uniform(0.8, 1.2, size=(inp.n, 2))
    v = rng.standard_normal(y.shape) * y
    exp, _ = o.year(u, y)
    ephi, ejv = o.year_tangent(u, y, v)
    out = {}
    for wl in (1, 0):
        t.set_option(tmm.TMM_OPT_WAVE_LOCAL, wl)
        assert t.query(tmm.TMM_Q_PERSISTENT) == 1
        assert t.query(tmm.TMM_Q_WAVE_LOCAL) == wl
        got, _ = t.year(t.state(y))
        phi, jv = t.year_jvp(t.state(y), t.state(v), mode=tmm.TMM_JVP_TANGENT)
        got, jv = got.cpu().numpy(), jv.cpu().numpy()
        assert pointwise(got, exp, 2, f"columns wave_local={wl}, one year") <= YEAR
        assert columnwise(jv, ejv, 2, f"columns wave_local={wl}, tangent") <= TANGENT
        out[wl] = (got, jv)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
