"""GPU parity: libtmm (through its C ABI) against the CPU oracle, same seeded inputs.

Tolerances (measured as in ``tolerances.py``: states point by point, signed
fields per tracer column, gradients per component): one step 1e-14, one
model year 1e-12 (the forward bar), the tangent 1e-11, the adjoint's dJ/du
and dJ/dy0 1e-10, J 1e-12 per member.
"""

import numpy as np
import pytest

import oracle
import synth
from tolerances import ADJOINT, FD, MISFIT, STEP, TANGENT, YEAR, columnwise, componentwise, pointwise

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1410_0204_amd import tmm
    return tmm


def _make(inp, nbatch_max=1, adjoint=0, ckpt=240):
    tmm = _lib()
    print(f"[gpu] create {inp.name} nbatch_max={nbatch_max} adjoint={adjoint}", flush=True)
    return tmm.TMM(inp.desc_arrays(), nbatch_max=nbatch_max, adjoint_nbatch_max=adjoint, ckpt_every=ckpt)


@pytest.fixture(scope="module")
def inputs():
    return {"tiny_n": synth.tiny(), "tiny_ndop": synth.tiny(model=synth.MODEL_NDOP),
            "small": synth.small_ndop()}


@pytest.mark.parametrize("name", ["tiny_n", "tiny_ndop", "small"])
def test_step_parity(inputs, name):
    inp = inputs[name]
    t = _make(inp)
    o = oracle.Oracle(inp)
    u = synth.nominal(inp.model)
    t.set_params(u)
    rng = np.random.default_rng(1)
    y = inp.initial_state() * rng.uniform(0.5, 1.5, size=(inp.n, inp.ntracer))
    yd = t.state(y)
    for j in (0, 119, 120, 1439, 2879):
        got = t.step(j, yd).cpu().numpy()
        exp = o.step(u, j, y)
        assert pointwise(got, exp, inp.ntracer, f"{name} step {j}") <= STEP, j


@pytest.mark.parametrize("name", ["tiny_n", "tiny_ndop", "small"])
def test_year_parity(inputs, name):
    inp = inputs[name]
    t = _make(inp)
    o = oracle.Oracle(inp)
    u = synth.nominal(inp.model)
    t.set_params(u)
    y0 = inp.initial_state()
    got, r = t.year(t.state(y0), nyears=2)
    exp, re = o.year(u, y0, 2)
    assert pointwise(got.cpu().numpy(), exp, inp.ntracer, f"{name} two years") <= YEAR
    assert np.allclose(r, re, rtol=1e-9, atol=0)


def test_batched_members_match_unbatched(inputs):
    inp = inputs["small"]
    U = synth.latin_hypercube(synth.MODEL_NDOP, 3, seed=2)
    t = _make(inp, nbatch_max=3)
    y0 = inp.initial_state(3)
    t.set_params(U)
    yb, rb = t.year(t.state(y0))
    yb = yb.cpu().numpy()
    for m in range(3):
        t.set_params(U[m])
        ym, rm = t.year(t.state(y0[:, 2 * m:2 * m + 2]))
        assert pointwise(ym.cpu().numpy(), yb[:, 2 * m:2 * m + 2], 2, f"member {m} alone vs batched") <= STEP
        assert rm[0, 0] == pytest.approx(rb[0, m], rel=1e-14)


@pytest.mark.parametrize("nb,nsteps", [(8, 2880), (70, 24)])
def test_member_parallel_kernel(inputs, nb, nsteps):
    """Ensembles through the member-parallel step kernel (two member groups, ragged) vs the oracle."""
    tmm = _lib()
    inp = inputs["small"]
    U = synth.latin_hypercube(synth.MODEL_NDOP, nb, seed=nb)
    t = _make(inp, nbatch_max=nb)
    t.set_option(tmm.TMM_OPT_MEMBER_KERNEL_MIN, 1)
    o = oracle.Oracle(inp)
    t.set_params(U)
    rng = np.random.default_rng(nb)
    y0 = inp.initial_state(nb) * rng.uniform(0.7, 1.3, size=(inp.n, 2 * nb))
    if nsteps == 2880:
        got, _ = t.year(t.state(y0))
        exp, _ = o.year(U, y0)
        assert pointwise(got.cpu().numpy(), exp, 2, f"{nb} members, one year") <= YEAR
    else:
        yd, ye = t.state(y0), y0
        for j in range(nsteps):
            yd = t.step(j * 119 % 2880, yd)
            ye = o.step(U, j * 119 % 2880, ye)
            assert pointwise(yd.cpu().numpy(), ye, 2, f"{nb} members, step {j}" if j == nsteps - 1 else None) <= STEP, j


@pytest.mark.parametrize("waves", [2, 4, 8])
def test_member_kernel_orders_and_waves(inputs, waves):
    """The member-parallel kernel with 2, 4 or 8 wavefronts per workgroup and each column order
    (natural, and bands of 1, 4 and 16 latitude rows swept by longitude, cut into one run per XCD)
    gives the oracle's step; every order gives the same result bit for bit (each column is computed
    the same way, only by another wavefront)."""
    tmm = _lib()
    inp = inputs["small"]
    nb = 70                                            # two member groups, the second ragged
    U = synth.latin_hypercube(synth.MODEL_NDOP, nb, seed=71)
    t = _make(inp, nbatch_max=nb)
    t.set_option(tmm.TMM_OPT_MEMBER_KERNEL_MIN, 1)
    t.set_option(tmm.TMM_OPT_MEMBER_WAVES, waves)
    t.set_params(U)
    rng = np.random.default_rng(72)
    y = inp.initial_state(nb) * rng.uniform(0.7, 1.3, size=(inp.n, 2 * nb))
    exp = oracle.Oracle(inp).step(U, 1439, y)
    ref = None
    for band in (-1, 1, 4, 16):
        t.set_option(tmm.TMM_OPT_MEMBER_BAND_ROWS, band)
        got = t.step(1439, t.state(y)).cpu().numpy()
        if ref is None:
            assert pointwise(got, exp, 2, f"{waves} waves, natural order") <= STEP
            ref = got
        else:
            assert np.array_equal(got, ref), band


@pytest.mark.parametrize("tile", [4, 8])
def test_member_tile_kernel(inputs, tile):
    """The tiled member kernel (workgroups of 4 or 8 neighbouring columns that stage each state row
    once per layer in LDS) gives the oracle's step, and the one-column-per-wavefront kernel's result
    bit for bit: at the start of the year, at a month boundary and at the year's last step, for two
    member groups (the second ragged) and for the kernel's smallest batch (6 members)."""
    tmm = _lib()
    inp = inputs["small"]
    o = oracle.Oracle(inp)
    for nb in (70, 6):
        U = synth.latin_hypercube(synth.MODEL_NDOP, nb, seed=73 + nb)
        t = _make(inp, nbatch_max=nb)
        t.set_params(U)
        rng = np.random.default_rng(74 + nb)
        y = inp.initial_state(nb) * rng.uniform(0.7, 1.3, size=(inp.n, 2 * nb))
        yd = t.state(y)
        for j in (0, 239, 240, 2879):
            ref = t.step(j, yd).cpu().numpy()
            t.set_option(tmm.TMM_OPT_MEMBER_BAND_ROWS, 2)
            t.set_option(tmm.TMM_OPT_MEMBER_TILE, tile)
            got = t.step(j, yd).cpu().numpy()
            t.set_option(tmm.TMM_OPT_MEMBER_TILE, 0)
            t.set_option(tmm.TMM_OPT_MEMBER_BAND_ROWS, 0)
            assert pointwise(got, o.step(U, j, y), 2, f"tile {tile}, {nb} members, step {j}") <= STEP, j
            assert np.array_equal(got, ref), (nb, j)
        t.close()


def test_member_tile_kernel_year_and_refusals(inputs):
    """Model years of an uneven ensemble on the tiled member kernel (graph-captured steps, members
    compacted as they finish) equal the oracle's years member by member; the option is refused where
    the kernel cannot run (one tracer, no band order) and leaves the handle as it was."""
    tmm = _lib()
    inp = inputs["small"]
    nb = 8
    U = synth.latin_hypercube(synth.MODEL_NDOP, nb, seed=81)
    L = np.array([2, 1, 2, 0, 1, 2, 2, 1], dtype=np.int32)
    t = _make(inp, nbatch_max=nb)
    t.set_params(U)
    t.set_option(tmm.TMM_OPT_MEMBER_BAND_ROWS, 2)
    t.set_option(tmm.TMM_OPT_MEMBER_TILE, 8)
    y0 = inp.initial_state(nb)
    got, _ = t.year(t.state(y0), nyears=2, years_per_member=L)
    got = got.cpu().numpy()
    o = oracle.Oracle(inp)
    for m in range(nb):
        exp = o.year(U[m], y0[:, 2 * m:2 * m + 2], int(L[m]))[0] if L[m] else y0[:, 2 * m:2 * m + 2]
        assert pointwise(got[:, 2 * m:2 * m + 2], exp, 2, f"tiled member kernel, member {m}") <= YEAR, m
    with pytest.raises(tmm.TmmError):
        t.set_option(tmm.TMM_OPT_MEMBER_BAND_ROWS, -1)      # tiles need the band order
    with pytest.raises(tmm.TmmError):
        t.set_option(tmm.TMM_OPT_MEMBER_TILE, 6)
    again, _ = t.year(t.state(y0), nyears=2, years_per_member=L)
    assert np.array_equal(again.cpu().numpy(), got)
    t.close()
    t1 = _make(inputs["tiny_n"], nbatch_max=8)
    with pytest.raises(tmm.TmmError):
        t1.set_option(tmm.TMM_OPT_MEMBER_TILE, 8)
    t1.close()


@pytest.mark.parametrize("nb", [2, 6, 16, 17, 32])
def test_packed_member_kernel(inputs, nb):
    """Batches of at most 32 (16) members run the member kernel with 2 (4) water columns per
    wavefront (from 2 members on by default): the oracle's step, and bit for bit the
    one-column-per-wavefront result, in the band order and in the natural order."""
    tmm = _lib()
    inp = inputs["small"]
    U = synth.latin_hypercube(synth.MODEL_NDOP, nb, seed=90 + nb)
    t = _make(inp, nbatch_max=nb)
    t.set_params(U)
    rng = np.random.default_rng(91 + nb)
    y = inp.initial_state(nb) * rng.uniform(0.7, 1.3, size=(inp.n, 2 * nb))
    yd = t.state(y)
    o = oracle.Oracle(inp)
    for band in (0, -1):
        t.set_option(tmm.TMM_OPT_MEMBER_BAND_ROWS, band)
        for j in (0, 1439, 2879):
            t.set_option(tmm.TMM_OPT_MEMBER_PACK, 0)
            t.set_option(tmm.TMM_OPT_MEMBER_KERNEL_MIN, 1)      # one column per wavefront at any width
            ref = t.step(j, yd).cpu().numpy()
            t.set_option(tmm.TMM_OPT_MEMBER_KERNEL_MIN, -1)     # the default crossover
            t.set_option(tmm.TMM_OPT_MEMBER_PACK, 1)
            got = t.step(j, yd).cpu().numpy()
            assert pointwise(got, o.step(U, j, y), 2, f"packed, {nb} members, band {band}, step {j}") <= STEP
            assert np.array_equal(got, ref), (band, j)
    t.close()


def test_uneven_spinup_lengths(inputs):
    """Members stop after their own number of years; finished states are kept."""
    inp = inputs["tiny_ndop"]
    U = synth.latin_hypercube(synth.MODEL_NDOP, 4, seed=5)
    L = np.array([2, 0, 1, 3], dtype=np.int32)
    t = _make(inp, nbatch_max=4)
    o = oracle.Oracle(inp)
    t.set_params(U)
    y0 = inp.initial_state(4)
    got, r = t.year(t.state(y0), nyears=3, years_per_member=L)
    got = got.cpu().numpy()
    for m in range(4):
        exp, re = o.year(U[m], y0[:, 2 * m:2 * m + 2], int(L[m])) if L[m] else (y0[:, 2 * m:2 * m + 2], None)
        assert pointwise(got[:, 2 * m:2 * m + 2], exp, 2, f"member {m}, {L[m]} years") <= YEAR, m
        if L[m]:
            assert np.allclose(r[:L[m], m], re[:, 0], rtol=1e-9)
            assert (r[L[m]:, m] == 0).all()


def test_jvp_tangent_and_fd(inputs):
    inp = inputs["small"]
    t = _make(inp)
    o = oracle.Oracle(inp)
    u = synth.nominal(inp.model)
    t.set_params(u)
    rng = np.random.default_rng(3)
    y = inp.initial_state() * rng.uniform(0.8, 1.2, size=(inp.n, 2))
    v = rng.standard_normal(y.shape) * y
    tmm = _lib()
    phi, jv = t.year_jvp(t.state(y), t.state(v), mode=tmm.TMM_JVP_TANGENT)
    ephi, ejv = o.year_tangent(u, y, v)
    assert pointwise(phi.cpu().numpy(), ephi, 2, "phi (tangent call)") <= YEAR
    assert columnwise(jv.cpu().numpy(), ejv, 2, "tangent") <= TANGENT
    phi, jfd = t.year_jvp(t.state(y), t.state(v), mode=tmm.TMM_JVP_FD)
    _, efd = o.year_jvp_fd(u, y, v)
    assert pointwise(phi.cpu().numpy(), ephi, 2, "phi (FD call)") <= YEAR
    # both are forward differences with h = 1e-8 |y|/|v|; rounding makes them agree to ~1e-6
    assert columnwise(jfd.cpu().numpy(), efd, 2, "FD vs oracle FD") <= FD
    assert columnwise(jfd.cpu().numpy(), ejv, 2, "FD vs oracle tangent") <= FD


@pytest.mark.parametrize("persistent", [1, 0])
@pytest.mark.parametrize("name,ckpt", [("tiny_n", 240), ("tiny_ndop", 240), ("small", 480), ("small", 1),
                                       ("tiny_ndop", 2880), ("small", 2880)])
def test_adjoint_parity(inputs, name, ckpt, persistent):
    inp = inputs[name]
    o = oracle.Oracle(inp)
    ustar = synth.hidden_params(inp.model, seed=21)
    y0 = inp.initial_state()
    snaps = o.snapshots(ustar, y0)
    obs = snaps * (1 + 0.05 * synth.obs_noise(snaps.shape, seed=22))
    u = synth.nominal(inp.model)
    eJ, eG, eY = o.year_adjoint(u, y0, obs)
    t = _make(inp, adjoint=1, ckpt=ckpt)
    t.set_option(_lib().TMM_OPT_PERSISTENT, persistent)
    t.set_params(u)
    import torch
    J, G, dy0 = t.year_adjoint(t.state(y0), torch.as_tensor(obs).cuda())
    assert componentwise(J, eJ, f"{name} ckpt {ckpt} J") <= MISFIT
    assert componentwise(G, eG, f"{name} ckpt {ckpt} dJ/du") <= ADJOINT
    assert columnwise(dy0.cpu().numpy(), eY, inp.ntracer, f"{name} ckpt {ckpt} dJ/dy0") <= ADJOINT


@pytest.mark.parametrize("name", ["tiny_n", "tiny_ndop", "small"])
def test_persistent_and_per_step_paths_agree(inputs, name):
    """The single-launch year kernel and the per-step kernels give the oracle's year."""
    tmm = _lib()
    inp = inputs[name]
    t = _make(inp)
    assert t.query(tmm.TMM_Q_PERSISTENT) == 1
    o = oracle.Oracle(inp)
    u = synth.nominal(inp.model)
    t.set_params(u)
    y0 = inp.initial_state()
    exp, _ = o.year(u, y0)
    out = {}
    for pers in (1, 0):
        t.set_option(tmm.TMM_OPT_PERSISTENT, pers)
        got, _ = t.year(t.state(y0))
        out[pers] = got.cpu().numpy()
        assert pointwise(out[pers], exp, inp.ntracer, f"{name} path {pers}") <= YEAR, pers
    assert pointwise(out[1], out[0], inp.ntracer) <= YEAR


@pytest.mark.parametrize("rows", [16, 32, 64, 256, 512])
def test_persistent_domain_sizes(inputs, rows):
    """Every domain partition (and so every dependency pattern) gives the same year."""
    tmm = _lib()
    inp = inputs["small"]
    t = _make(inp)
    t.set_option(tmm.TMM_OPT_DOMAIN_ROWS, rows)
    print(f"[gpu] domains: {t.query(tmm.TMM_Q_DOMAINS)}", flush=True)
    o = oracle.Oracle(inp)
    u = synth.nominal(inp.model)
    t.set_params(u)
    y0 = inp.initial_state()
    got, _ = t.year(t.state(y0), nyears=2)
    exp, _ = o.year(u, y0, 2)
    assert pointwise(got.cpu().numpy(), exp, 2, f"{rows} rows, two years") <= YEAR
    rng = np.random.default_rng(7)
    v = rng.standard_normal(y0.shape)
    phi, jv = t.year_jvp(t.state(y0), t.state(v), mode=tmm.TMM_JVP_TANGENT)
    ephi, ejv = o.year_tangent(u, y0, v)
    assert pointwise(phi.cpu().numpy(), ephi, 2) <= YEAR
    assert columnwise(jv.cpu().numpy(), ejv, 2, f"{rows} rows, tangent") <= TANGENT


@pytest.mark.parametrize("nb", [1, 3, 20])
def test_graph_replays_match_eager(inputs, nb):
    """Model years replayed from captured graphs equal eager launches bitwise, replay after replay,
    with other work on the stream in between."""
    tmm = _lib()
    inp = inputs["small"]
    U = synth.latin_hypercube(synth.MODEL_NDOP, nb, seed=40 + nb)
    t = _make(inp, nbatch_max=nb)
    t.set_option(tmm.TMM_OPT_PERSISTENT, 0)
    t.set_params(U)
    y0 = t.state(inp.initial_state(nb))
    t.set_option(tmm.TMM_OPT_GRAPH, 0)
    e1, r1 = t.year(y0)
    e2, r2 = t.year(e1)
    t.set_option(tmm.TMM_OPT_GRAPH, 1)
    for rep in range(3):
        g1, q1 = t.year(y0)
        t.step(rep * 7, g1)                 # eager work between replays
        g2, q2 = t.year(g1)
        assert bool((g1 == e1).all()) and bool((g2 == e2).all()), rep
        assert np.array_equal(q1, r1) and np.array_equal(q2, r2)


def test_year_is_deterministic(inputs):
    inp = inputs["small"]
    t = _make(inp)
    t.set_params(synth.nominal(inp.model))
    y0 = t.state(inp.initial_state())
    a, _ = t.year(y0)
    b, _ = t.year(y0)
    assert bool((a == b).all())


@pytest.fixture(scope="module")
def global_inputs():
    return synth.global_2p8()


def test_global_step_and_year_parity(global_inputs):
    """Full 128x64x15 workload (52749 points, N-DOP) in the benchmark's launch configuration."""
    inp = global_inputs
    t = _make(inp)
    tmm = _lib()
    assert t.query(tmm.TMM_Q_PERSISTENT) == 1
    print(f"[gpu] global: {t.query(tmm.TMM_Q_DOMAINS)} domains on {t.query(tmm.TMM_Q_COMPUTE_UNITS)} CUs", flush=True)
    o = oracle.Oracle(inp)
    u = synth.nominal(inp.model)
    t.set_params(u)
    y0 = inp.initial_state()
    yd = t.state(y0)
    for j in (0, 2879):
        assert pointwise(t.step(j, yd).cpu().numpy(), o.step(u, j, y0), 2, f"global step {j}") <= STEP
    print("[gpu] global year on the oracle (~15 s)", flush=True)
    got, r = t.year(yd)
    exp, re = o.year(u, y0)
    assert pointwise(got.cpu().numpy(), exp, 2, "global year") <= YEAR
    assert r[0, 0] == pytest.approx(re[0, 0], rel=1e-9)
