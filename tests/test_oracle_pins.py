"""Pins of the reference implementation against facts fixed outside it.

Each test checks the oracle against something it does not compute itself:
closed forms that follow from the paper's formulas, invariants of the
transport (row-stochastic, volume-conserving matrices), brute force on tiny
inputs, numerical quadrature, and finite differences.  A plausible mistake in
the oracle (a dropped term, a wrong sign, a transposed operand, an off-by-one
in the month interpolation, a wrong depth for the light) fails at least one.
"""

import math

import numpy as np
import pytest

import oracle
import synth

S0 = 1361.0
SIGMA_PAR = 0.4


# --------------------------------------------------------------------------
# Month interpolation (section 3; mid-month anchors, periodic year)
# --------------------------------------------------------------------------

def _phase_by_month_centres(j, nstep=2880, nmat=12):
    """Independent restatement: matrices sit at month centres (k+1/2)/nmat."""
    t = j / nstep
    centres = (np.arange(nmat) + 0.5) / nmat
    # last centre at or before t, wrapping to December before mid-January
    before = np.nonzero(centres <= t + 1e-15)[0]
    k0 = int(before[-1]) if before.size else nmat - 1
    t0 = centres[k0] if before.size else centres[-1] - 1.0
    return k0, (k0 + 1) % nmat, (t - t0) * nmat


def test_phase_anchor_points():
    assert oracle.phase(0) == (11, 0, 0.5)
    assert oracle.phase(120) == (0, 1, 0.0)
    assert oracle.phase(119) == (11, 0, 239 / 240)
    assert oracle.phase(2879) == (11, 0, 119 / 240)
    assert oracle.phase(2880) == oracle.phase(0)
    assert oracle.phase(360) == (1, 2, 0.0)


def test_phase_matches_month_centres_everywhere():
    for j in range(2880):
        k0, k1, w = oracle.phase(j)
        e0, e1, ew = _phase_by_month_centres(j)
        assert (k0, k1) == (e0, e1)
        assert abs(w - ew) < 1e-12
        assert w == round(w * 240) / 240            # exact integer phase r/240


# --------------------------------------------------------------------------
# Insolation (section 2.2.1; daily-mean top-of-atmosphere formula)
# --------------------------------------------------------------------------

def _declination(t):
    return math.radians(-23.44) * math.cos(2 * math.pi * (t + 10 / 360))


def _insolation_quadrature(lat, t, m=20000):
    """Average over the day of S0 * max(0, cos(zenith)) by the midpoint rule."""
    phi, d = math.radians(lat), _declination(t)
    h = -math.pi + (np.arange(m) + 0.5) * 2 * math.pi / m
    mu = math.sin(phi) * math.sin(d) + math.cos(phi) * math.cos(d) * np.cos(h)
    return S0 * np.maximum(mu, 0).mean()


def test_insolation_closed_forms():
    t_equinox = 0.25 - 10 / 360                      # declination zero
    assert oracle.insolation(0.0, t_equinox) == pytest.approx(S0 / math.pi, rel=1e-12)
    assert oracle.insolation(80.0, 0.0) == 0.0       # polar night in northern winter
    assert oracle.insolation(-80.0, 0.0) > 0.0       # polar day in southern summer
    for lat in (-75.0, -33.0, 0.0, 12.5, 61.0):
        for t in (0.0, 0.13, 0.4, 0.77):
            q = oracle.insolation(lat, t)
            assert 0.0 <= q <= S0
            assert q == pytest.approx(oracle.insolation(-lat, t + 0.5), rel=1e-12, abs=1e-9)


@pytest.mark.parametrize("lat,t", [(0.0, 0.0), (45.0, 0.3), (-60.0, 0.1), (70.0, 0.5), (-88.6, 0.0)])
def test_insolation_matches_quadrature(lat, t):
    assert oracle.insolation(lat, t) == pytest.approx(_insolation_quadrature(lat, t), rel=1e-6, abs=1e-6)


# --------------------------------------------------------------------------
# Biogeochemical model of one column (section 2.2.1)
# --------------------------------------------------------------------------

U_NDOP = synth.nominal(synth.MODEL_NDOP)   # alpha, K_H2O, K1, K_I, lambda2, sigma2, b
U_N = synth.nominal(synth.MODEL_N)         # alpha, K_H2O, K_N, K_I, b


def test_production_half_saturation_and_light_ratio():
    """With N = K1 and I_0 = K_I, f_0 = alpha/4; choosing K_H2O with I_1/I_0 = 1/3 gives f_1 = alpha/8."""
    h = np.array([50.0, 80.0, 300.0, 400.0])
    z0, z1 = h[0] / 2, h[0] + h[1] / 2
    u = U_NDOP.copy()
    u[1] = math.log(3.0) / (z1 - z0)             # K_H2O
    insol = u[3] / (SIGMA_PAR * math.exp(-z0 * u[1]))
    y = np.zeros((2, 4))
    y[0, :] = u[2]                                 # PO4 = K1 everywhere, DOP = 0
    q = oracle.bgc_column(synth.MODEL_NDOP, insol, h, y, u, neuphotic=2)
    alpha, sigma = u[0], u[5]
    # euphotic layers: PO4 consumed by f, DOP gains sigma*f
    assert -q[0, 0] == pytest.approx(alpha / 4, rel=1e-14)
    assert -q[0, 1] == pytest.approx(alpha / 8, rel=1e-14)
    assert q[1, 0] == pytest.approx(sigma * alpha / 4, rel=1e-14)
    assert q[1, 1] == pytest.approx(sigma * alpha / 8, rel=1e-14)


def test_martin_curve_closed_form():
    """h = [l'/2, l'/2, l', l', l'] puts the aphotic interfaces at l', 2l', 3l'."""
    lp = 120.0
    h = np.array([lp / 2, lp / 2, lp, lp, lp])
    b = 0.9
    u = U_N.copy()
    u[4] = b
    y = np.full((1, 5), 1.3)
    q = oracle.bgc_column(synth.MODEL_N, 250.0, h, y, u, neuphotic=2)
    Phi = -(h[0] * q[0, 0] + h[1] * q[0, 1])      # export = production integral
    assert Phi > 0
    assert q[0, 2] == pytest.approx(Phi * (1 - 2 ** -b) / lp, rel=1e-13)
    assert q[0, 3] == pytest.approx(Phi * (2 ** -b - 3 ** -b) / lp, rel=1e-13)
    assert q[0, 4] == pytest.approx(Phi * 3 ** -b / lp, rel=1e-13)   # sea floor keeps the rest
    assert (h * q[0]).sum() == pytest.approx(0.0, abs=1e-15 * Phi)


def test_column_mass_balance_and_dop_terms():
    rng = np.random.default_rng(0)
    h = synth.grid.layer_heights(15)
    for nl in (1, 2, 3, 9, 15):
        y = rng.uniform(0.1, 3.0, size=(2, nl))
        u = synth.latin_hypercube(synth.MODEL_NDOP, 1, seed=nl)[0]
        q = oracle.bgc_column(synth.MODEL_NDOP, 300.0, h, y, u, neuphotic=2)
        total = (h[:nl] * (q[0] + q[1])).sum()
        scale = (h[:nl] * np.abs(q).sum(0)).sum()
        assert abs(total) <= 1e-14 * scale
    # no light: only DOP remineralisation, exactly lambda*DOP moved back to PO4
    y = rng.uniform(0.1, 3.0, size=(2, 6))
    q = oracle.bgc_column(synth.MODEL_NDOP, 0.0, h, y, U_NDOP, neuphotic=2)
    assert np.array_equal(q[1], -U_NDOP[4] * y[1])
    assert np.allclose(q[0], U_NDOP[4] * y[1], rtol=1e-15, atol=0)


def test_shallow_column_exports_to_bottom():
    """A column no deeper than the euphotic zone remineralises its export in its bottom layer."""
    h = np.array([40.0, 60.0, 500.0])
    q = oracle.bgc_column(synth.MODEL_N, 200.0, h, np.array([[1.0]]), U_N, neuphotic=2)
    assert abs(q[0, 0]) < 1e-16                      # one layer: produced and returned in place
    q = oracle.bgc_column(synth.MODEL_N, 200.0, h, np.array([[1.0, 1.0]]), U_N, neuphotic=2)
    # q_0 = -f_0 and q_1 = -f_1 + (h_0 f_0 + h_1 f_1)/h_1 = h_0 f_0 / h_1
    assert q[0, 0] < 0
    assert q[0, 1] == pytest.approx(-h[0] * q[0, 0] / h[1], rel=1e-14)


# --------------------------------------------------------------------------
# Transport: invariants and brute force
# --------------------------------------------------------------------------

def _dense_month(tm, kind, m, n):
    rowptr = getattr(tm, kind + "_rowptr")
    colidx = getattr(tm, kind + "_colidx")
    val = getattr(tm, kind + "_val")[m]
    A = np.zeros((n, n))
    for i in range(n):
        for e in range(rowptr[i], rowptr[i + 1]):
            A[i, colidx[e]] += val[e]
    return A


def _dense_interp(inp, j, kind, dense_cache):
    k0, k1, w = _phase_by_month_centres(j, inp.nstep, inp.nmat)
    A0 = dense_cache[(kind, k0)]
    A1 = dense_cache[(kind, k1)]
    return (1 - w) * A0 + w * A1


@pytest.fixture(scope="module")
def tiny_dense(tiny_n):
    n = tiny_n.n
    cache = {}
    for kind in ("ae", "ai"):
        for m in range(tiny_n.nmat):
            cache[(kind, m)] = _dense_month(tiny_n.tm, kind, m, n)
    return cache


def test_linear_year_map_dense_brute_force(tiny_n, tiny_dense):
    """alpha = 0 removes the BGC: phi(y) = prod_j Ai(t_j) Ae(t_j) y, built densely."""
    n = tiny_n.n
    M = np.eye(n)
    for j in range(tiny_n.nstep):
        M = _dense_interp(tiny_n, j, "ai", tiny_dense) @ (_dense_interp(tiny_n, j, "ae", tiny_dense) @ M)
    V = tiny_n.grid.volumes()
    assert np.abs(M @ np.ones(n) - 1).max() < 1e-12
    assert np.abs(V @ M - V).max() < 1e-12 * V.max()
    u = U_N.copy()
    u[0] = 0.0
    y0 = np.random.default_rng(1).uniform(0.5, 3.0, size=(n, 1))
    y1, _ = oracle.Oracle(tiny_n).year(u, y0)
    assert np.abs(y1 - M @ y0).max() <= 1e-12 * np.abs(y0).max()


def test_one_step_dense_with_bgc(tiny_ndop):
    """One step with the BGC on: Ai (Ae y + dt_d q) assembled densely from column calls."""
    inp = tiny_ndop
    n, g = inp.n, inp.grid
    dense = {(k, m): _dense_month(inp.tm, k, m, n) for k in ("ae", "ai") for m in range(inp.nmat)}
    o = oracle.Oracle(inp)
    rng = np.random.default_rng(2)
    y = np.column_stack([rng.uniform(0.5, 3.0, n), rng.uniform(0.0, 0.2, n)])
    u = synth.nominal(synth.MODEL_NDOP)
    for j in (0, 77, 1439, 2879):
        t = j / inp.nstep
        q = np.zeros_like(y)
        for c in range(g.ncol):
            s, e = g.col_start[c], g.col_start[c + 1]
            insol = oracle.insolation(g.lat[c], t)
            q[s:e] = oracle.bgc_column(inp.model, insol, g.dz, y[s:e].T, u, inp.neuphotic).T
        Ae = _dense_interp(inp, j, "ae", dense)
        Ai = _dense_interp(inp, j, "ai", dense)
        expect = Ai @ (Ae @ y + (360.0 / inp.nstep) * q)
        got = o.step(u, j, y)
        assert np.abs(got - expect).max() <= 1e-14 * np.abs(expect).max()


def test_constant_field_preserved_without_bgc(small_ndop):
    u = synth.nominal(synth.MODEL_NDOP)
    u[0] = 0.0          # no production
    u[4] = 0.0          # no DOP remineralisation: q == 0
    o = oracle.Oracle(small_ndop)
    y0 = np.column_stack([np.full(small_ndop.n, 2.17), np.full(small_ndop.n, 0.3)])
    y1, resid = o.year(u, y0)
    assert np.abs(y1 / y0 - 1).max() < 2e-13
    assert resid[0, 0] < 1e-10


def test_mass_conserved_and_positive_with_bgc(small_ndop):
    u = synth.nominal(synth.MODEL_NDOP)
    o = oracle.Oracle(small_ndop)
    y0 = small_ndop.initial_state()
    y1, _ = o.year(u, y0)
    V = small_ndop.grid.volumes()
    m0 = V @ (y0[:, 0] + y0[:, 1])
    m1 = V @ (y1[:, 0] + y1[:, 1])
    assert abs(m1 - m0) <= 1e-13 * m0
    assert y1.min() > 0.0
    assert np.abs(y1 - y0).max() > 1e-3     # the BGC did something


def test_identity_transport_decay_closed_form(tiny_ndop):
    """Ae = Ai = I and alpha = 0: DOP_j = (1 - lambda dt_d)^j DOP_0 and PO4 + DOP is constant."""
    inp = tiny_ndop
    tm = inp.tm
    import copy
    ident = copy.deepcopy(inp)
    for kind in ("ae", "ai"):
        rowptr = getattr(tm, kind + "_rowptr")
        colidx = getattr(tm, kind + "_colidx")
        rows = np.repeat(np.arange(inp.n), np.diff(rowptr))
        val = np.where(rows == colidx, 1.0, 0.0)
        setattr(ident.tm, kind + "_val", np.broadcast_to(val, (inp.nmat, val.size)).copy())
    u = synth.nominal(synth.MODEL_NDOP)
    u[0] = 0.0
    o = oracle.Oracle(ident)
    y0 = np.column_stack([np.full(inp.n, 2.0), np.linspace(0.1, 0.5, inp.n)])
    y1, _ = o.year(u, y0)
    dtd = 360.0 / inp.nstep
    decay = (1 - u[4] * dtd) ** inp.nstep
    assert np.abs(y1[:, 1] / (y0[:, 1] * decay) - 1).max() < 2e-13   # 2880 roundings
    assert np.abs(y1.sum(1) / y0.sum(1) - 1).max() < 2e-13


def test_restart_is_bitwise(tiny_ndop):
    o = oracle.Oracle(tiny_ndop)
    u = synth.nominal(synth.MODEL_NDOP)
    y0 = tiny_ndop.initial_state()
    a, _ = o.year(u, y0, 1)
    a, _ = o.year(u, a, 1)
    b, r = o.year(u, y0, 2)
    assert np.array_equal(a, b)
    c, _ = o.year(u, y0, 1)
    assert r[0, 0] == pytest.approx(np.linalg.norm(c - y0), rel=1e-14)
    assert r[1, 0] == pytest.approx(np.linalg.norm(b - c), rel=1e-14)


def test_batch_members_are_independent(tiny_ndop):
    o = oracle.Oracle(tiny_ndop)
    U = synth.latin_hypercube(synth.MODEL_NDOP, 3, seed=9)
    y0 = tiny_ndop.initial_state(3)
    y0[:, 2:4] *= 1.1
    yb, rb = o.year(U, y0)
    for m in range(3):
        ym, rm = o.year(U[m], y0[:, 2 * m:2 * m + 2])
        assert np.array_equal(ym, yb[:, 2 * m:2 * m + 2])
        assert rm[0, 0] == rb[0, m]


# --------------------------------------------------------------------------
# Derivatives: tangent, finite differences, reverse mode
# --------------------------------------------------------------------------

def test_tangent_exact_for_linear_map(tiny_ndop):
    """alpha = 0 makes phi linear with phi(0) = 0, so phi'(y) v = phi(v)."""
    o = oracle.Oracle(tiny_ndop)
    u = synth.nominal(synth.MODEL_NDOP)
    u[0] = 0.0
    rng = np.random.default_rng(3)
    y = tiny_ndop.initial_state()
    v = rng.standard_normal(y.shape)
    _, jv = o.year_tangent(u, y, v)
    pv, _ = o.year(u, v)
    assert np.abs(jv - pv).max() < 1e-13 * np.abs(pv).max()
    _, jfd = o.year_jvp_fd(u, y, v)
    # forward differences at h = 1e-8 ‖y‖/‖v‖ carry rounding error of order eps*‖y‖/h
    assert np.abs(jfd - pv).max() < 1e-5 * np.abs(pv).max()


def test_tangent_matches_central_differences(tiny_ndop):
    o = oracle.Oracle(tiny_ndop)
    u = synth.nominal(synth.MODEL_NDOP)
    rng = np.random.default_rng(4)
    y = tiny_ndop.initial_state() * rng.uniform(0.8, 1.2, size=(tiny_ndop.n, 2))
    v = rng.standard_normal(y.shape) * y
    phi, jv = o.year_tangent(u, y, v)
    h = 1e-5
    yp, _ = o.year(u, y + h * v)
    ym, _ = o.year(u, y - h * v)
    fd = (yp - ym) / (2 * h)
    assert np.abs(jv - fd).max() < 1e-7 * np.abs(jv).max()
    p2, _ = o.year(u, y)
    assert np.array_equal(phi, p2)


def test_dot_product_tangent_vs_reverse(tiny_ndop):
    """<w, phi'(y) v> = <phi'(y)^T w, v> with tangent and reverse computed independently."""
    o = oracle.Oracle(tiny_ndop)
    u = synth.nominal(synth.MODEL_NDOP)
    rng = np.random.default_rng(5)
    y = tiny_ndop.initial_state() * rng.uniform(0.8, 1.2, size=(tiny_ndop.n, 2))
    v = rng.standard_normal(y.shape)
    w = rng.standard_normal(y.shape)
    _, jv = o.year_tangent(u, y, v)
    ybar, _ = o.year_vjp(u, y, w)
    lhs, rhs = np.sum(w * jv), np.sum(ybar * v)
    assert lhs == pytest.approx(rhs, rel=1e-12)


def _obs(inp, seed=21):
    o = oracle.Oracle(inp)
    ustar = synth.hidden_params(inp.model, seed=seed)
    snaps = o.snapshots(ustar, inp.initial_state())
    return snaps * (1 + 0.05 * synth.obs_noise(snaps.shape, seed=seed + 1))


def _fd4(f, x, h):
    """Fourth-order central difference: truncation O(h^4), rounding O(eps*|f|/h)."""
    return (-f(x + 2 * h) + 8 * f(x + h) - 8 * f(x - h) + f(x - 2 * h)) / (12 * h)


@pytest.mark.parametrize("which", ["n", "ndop"])
def test_parameter_gradient_matches_central_differences(which, tiny_n, tiny_ndop):
    """dJ/du by reverse mode vs. fourth-order central differences of the misfit.

    The year map's rounding makes J noisy at about 1e-15 relative, so plain
    central differences with h = 1e-6 |u_p| carry up to ~1e-5 relative noise on
    the smallest gradient components; h = 1e-4 |u_p| with a fourth-order
    stencil keeps both truncation and rounding below 1e-7.
    """
    inp = tiny_n if which == "n" else tiny_ndop
    o = oracle.Oracle(inp)
    obs = _obs(inp)
    u = synth.nominal(inp.model)
    y0 = inp.initial_state()
    J, dJdu, _ = o.year_adjoint(u, y0, obs)
    assert J[0] == pytest.approx(o.year_misfit(u, y0, obs)[0], rel=1e-14)
    for p in range(u.size):
        def Jp(x):
            v = u.copy()
            v[p] = x
            return o.year_misfit(v, y0, obs)[0]
        fd = _fd4(Jp, u[p], 1e-4 * abs(u[p]))
        assert dJdu[0, p] == pytest.approx(fd, rel=1e-6), p


def test_initial_state_gradient_matches_central_differences(tiny_ndop):
    o = oracle.Oracle(tiny_ndop)
    obs = _obs(tiny_ndop)
    u = synth.nominal(synth.MODEL_NDOP)
    y0 = tiny_ndop.initial_state()
    _, _, g = o.year_adjoint(u, y0, obs)
    rng = np.random.default_rng(6)
    for _ in range(3):
        d = rng.standard_normal(y0.shape) * y0
        fd = _fd4(lambda s: o.year_misfit(u, y0 + s * d, obs)[0], 0.0, 1e-4)
        assert np.sum(g * d) == pytest.approx(fd, rel=1e-6)


# --------------------------------------------------------------------------
# The misfit itself: its volume weights and normalisation.  The gradient pins
# above check dJ/du and dJ/dy0 against differences of the oracle's own J, so
# a wrong cell volume would go unnoticed there (J and its source share it);
# here J is written out from the month-end states and the grid's geometry.
# --------------------------------------------------------------------------

def _volumes_from_desc(inp):
    """V_i = area_c h_k, straight from the descriptor arrays."""
    a = inp.desc_arrays()
    V = np.empty(a["n"])
    for c in range(a["ncol"]):
        r0, r1 = int(a["col_start"][c]), int(a["col_start"][c + 1])
        V[r0:r1] = a["area"][c] * a["dz"][: r1 - r0]
    return V


def _misfit_by_hand(states, obs, V, nmat):
    """J_b = sum_m sum_i sum_tr V_i (y - o)^2 / (2 nmat V_tot) for each member b."""
    d2 = (states - obs) ** 2                                  # [nmat, n, W]
    return np.einsum("i,miw->w", V, d2) / (2.0 * nmat * V.sum())


@pytest.mark.parametrize("which", ["n", "ndop", "small", "batch"])
def test_misfit_value_restated(which, tiny_n, tiny_ndop, small_ndop):
    inp = {"n": tiny_n, "ndop": tiny_ndop, "small": small_ndop, "batch": tiny_ndop}[which]
    o = oracle.Oracle(inp)
    nb = 2 if which == "batch" else 1
    u = synth.nominal(inp.model) if nb == 1 else synth.latin_hypercube(inp.model, nb, seed=9)
    y0 = inp.initial_state(nb)
    obs1 = _obs(inp)
    obs = np.concatenate([obs1, obs1 * 1.03], axis=2) if nb == 2 else obs1
    V = _volumes_from_desc(inp)
    assert np.array_equal(V, inp.grid.volumes())
    states = o.snapshots(u, y0)                               # after steps 240 (m + 1)
    per_col = _misfit_by_hand(states, obs, V, inp.nmat)
    J = per_col.reshape(nb, inp.ntracer).sum(axis=1)
    assert np.allclose(o.year_misfit(u, y0, obs), J, rtol=1e-14, atol=0)
    assert np.allclose(o.year_adjoint(u, y0, obs)[0], J, rtol=1e-14, atol=0)
    # the pin separates the plausible mistakes: uniform weights, the layer
    # heights of another column depth (reversed), no factor 1/2, V_tot of one layer
    top = np.zeros_like(V)
    top[inp.grid.col_start[:-1]] = V[inp.grid.col_start[:-1]]
    dz_rev = inp.desc_arrays()["dz"][::-1]
    V_rev = np.concatenate([inp.desc_arrays()["area"][c] * dz_rev[: inp.grid.col_start[c + 1] - inp.grid.col_start[c]]
                            for c in range(inp.grid.ncol)])
    for wrong in (_misfit_by_hand(states, obs, np.ones_like(V), inp.nmat),
                  _misfit_by_hand(states, obs, V_rev, inp.nmat),
                  2.0 * per_col,
                  per_col * V.sum() / top.sum()):
        Jw = wrong.reshape(nb, inp.ntracer).sum(axis=1)
        assert np.abs(Jw / J - 1.0).max() > 1e-3


# --------------------------------------------------------------------------
# Internal BGC steps (section 7: several biogeochemical steps per ocean step)
# --------------------------------------------------------------------------

def _column(inp, c):
    g = inp.grid
    return g.col_start[c], g.col_start[c + 1], g.lat[c]


def test_single_substep_is_the_plain_source(tiny_ndop):
    """nbgc = 1 (and 0) reproduce dt*q bitwise, so every other pin covers that path."""
    inp = tiny_ndop
    u = synth.nominal(synth.MODEL_NDOP)
    s, e, lat = _column(inp, 3)
    y = inp.initial_state()[s:e].T.copy()
    insol = oracle.insolation(lat, 0.2)
    dt = 360.0 / inp.nstep
    q = oracle.bgc_column(inp.model, insol, inp.grid.dz[:e - s], y, u, inp.neuphotic)
    inc = oracle.bgc_source(inp.model, insol, inp.grid.dz[:e - s], y, u, inp.neuphotic, dt, 1)
    assert np.array_equal(inc, dt * q)
    y0 = inp.initial_state()
    a, _ = oracle.Oracle(inp, nbgc=0).year(u, y0)
    b, _ = oracle.Oracle(inp, nbgc=1).year(u, y0)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("grid", ["tiny_ndop", "tiny_phy"])
def test_substeps_are_explicit_euler_of_the_column_ode(grid, request):
    """The source with n internal steps is n explicit Euler steps of dt/n on dy/dt = q(y).

    Brute force from the (separately pinned) column term, and first-order
    convergence towards a fine-step solution of the same ODE; for PO4-DOP and
    PO4-DOP-PHY."""
    inp = request.getfixturevalue(grid)
    u = synth.nominal(inp.model)
    dt = 360.0 / inp.nstep
    for c in (0, 40):
        s, e, lat = _column(inp, c)
        h = inp.grid.dz[:e - s]
        y0 = inp.initial_state()[s:e].T.copy()
        insol = oracle.insolation(lat, 0.45)

        def euler(n, step):
            y = y0.copy()
            for _ in range(n):
                y = y + step * oracle.bgc_column(inp.model, insol, h, y, u, inp.neuphotic)
            return y
        for step in (dt, 30.0):
            end = y0 + oracle.bgc_source(inp.model, insol, h, y0, u, inp.neuphotic, step, 8)
            assert np.abs(end - euler(8, step / 8)).max() <= 1e-14 * np.abs(y0).max()
        # first order: over a 5-day step the error against 8192 Euler steps halves as n doubles;
        # PO4-DOP-PHY's growth scales with PHY itself, so its first-order regime starts at
        # shorter sub-steps: a 1-day step there
        span, ns = (5.0, (4, 8, 16, 32)) if inp.model == synth.MODEL_NDOP else (1.0, (4, 8, 16))
        fine = euler(8192, span / 8192) - y0
        errs = [np.abs(oracle.bgc_source(inp.model, insol, h, y0, u, inp.neuphotic, span, n) - fine).max()
                for n in ns]
        assert errs[0] > 1e-6 * np.abs(fine).max()
        for a, b in zip(errs, errs[1:]):
            assert 1.8 < a / b < 2.2, errs


def test_substep_decay_closed_form(tiny_ndop):
    """Identity transport and alpha = 0: each ocean step multiplies DOP by (1 - lambda dt/n)^n."""
    import copy
    inp = tiny_ndop
    ident = copy.deepcopy(inp)
    for kind in ("ae", "ai"):
        rowptr = getattr(inp.tm, kind + "_rowptr")
        colidx = getattr(inp.tm, kind + "_colidx")
        rows = np.repeat(np.arange(inp.n), np.diff(rowptr))
        val = np.where(rows == colidx, 1.0, 0.0)
        setattr(ident.tm, kind + "_val", np.broadcast_to(val, (inp.nmat, val.size)).copy())
    u = synth.nominal(synth.MODEL_NDOP)
    u[0] = 0.0
    y0 = np.column_stack([np.full(inp.n, 2.0), np.linspace(0.1, 0.5, inp.n)])
    dtd = 360.0 / inp.nstep
    for nb in (2, 8):
        y1, _ = oracle.Oracle(ident, nbgc=nb).year(u, y0)
        decay = (1 - u[4] * dtd / nb) ** (nb * inp.nstep)
        assert np.abs(y1[:, 1] / (y0[:, 1] * decay) - 1).max() < 1e-12
        assert np.abs(y1.sum(1) / y0.sum(1) - 1).max() < 2e-13


@pytest.mark.parametrize("model", [synth.MODEL_NDOP, synth.MODEL_NDOPPHY])
def test_substeps_conserve_mass(small_ndop, model):
    inp = small_ndop if model == synth.MODEL_NDOP else synth.small_ndop(model=model)
    u = synth.nominal(model)
    y0 = inp.initial_state()
    y1, _ = oracle.Oracle(inp, nbgc=8).year(u, y0)
    y1p, _ = oracle.Oracle(inp, nbgc=1).year(u, y0)
    V = inp.grid.volumes()
    m0 = V @ y0.sum(1)
    assert abs(V @ y1.sum(1) - m0) <= 1e-13 * m0
    assert 0 < np.abs(y1 - y1p).max() < 0.05 * np.abs(y1p).max()   # close to, not equal to, one step


@pytest.mark.parametrize("grid", ["tiny_ndop", "tiny_phy"])
def test_substep_derivatives(grid, request):
    """Tangent vs central differences, tangent vs reverse (dot test), dJ/du vs differences, with nbgc = 8
    (PO4-DOP and PO4-DOP-PHY)."""
    inp = request.getfixturevalue(grid)
    o = oracle.Oracle(inp, nbgc=8)
    u = synth.nominal(inp.model)
    rng = np.random.default_rng(14)
    y = inp.initial_state() * rng.uniform(0.8, 1.2, size=(inp.n, inp.ntracer))
    v = rng.standard_normal(y.shape) * y
    w = rng.standard_normal(y.shape)
    _, jv = o.year_tangent(u, y, v)
    h = 1e-5
    fd = (o.year(u, y + h * v)[0] - o.year(u, y - h * v)[0]) / (2 * h)
    assert np.abs(jv - fd).max() < 1e-7 * np.abs(jv).max()
    ybar, _ = o.year_vjp(u, y, w)
    assert np.sum(w * jv) == pytest.approx(np.sum(ybar * v), rel=1e-12)
    obs = _obs(inp)
    y0 = inp.initial_state()
    J, dJdu, _ = o.year_adjoint(u, y0, obs)
    for p in range(u.size):
        def Jp(x):
            q = u.copy()
            q[p] = x
            return o.year_misfit(q, y0, obs)[0]
        assert dJdu[0, p] == pytest.approx(_fd4(Jp, u[p], 1e-4 * abs(u[p])), rel=1e-6), p


# --------------------------------------------------------------------------
# PO4-DOP-PHY (section 2.2.2)
# --------------------------------------------------------------------------

PHY = synth.MODEL_NDOPPHY


def _identity_transport(inp):
    import copy
    ident = copy.deepcopy(inp)
    for kind in ("ae", "ai"):
        rowptr = getattr(inp.tm, kind + "_rowptr")
        colidx = getattr(inp.tm, kind + "_colidx")
        rows = np.repeat(np.arange(inp.n), np.diff(rowptr))
        val = np.where(rows == colidx, 1.0, 0.0)
        setattr(ident.tm, kind + "_val", np.broadcast_to(val, (inp.nmat, val.size)).copy())
    return ident


@pytest.fixture(scope="module")
def tiny_phy():
    return synth.tiny(model=PHY)


def test_phy_column_conserves_phosphorus(tiny_phy):
    """sum_k h_k (q_PO4 + q_DOP + q_PHY) = 0 in every column: export, grazing and losses only move P."""
    inp = tiny_phy
    g = inp.grid
    rng = np.random.default_rng(20)
    u = synth.latin_hypercube(PHY, 1, seed=21)[0]
    checked = 0
    for c in range(g.ncol):
        s, e = g.col_start[c], g.col_start[c + 1]
        h = g.dz[:e - s]
        y = np.vstack([rng.uniform(0.5, 3.0, e - s), rng.uniform(0.0, 0.2, e - s), rng.uniform(0.0, 0.5, e - s)])
        q = oracle.bgc_column(PHY, 300.0, h, y, u, inp.neuphotic)
        scale = np.abs(q * h).max()
        assert abs(np.sum(q * h)) <= 1e-14 * scale * q.size, c
        checked += 1
    assert checked == g.ncol


def test_phy_reduces_to_po4_dop(tiny_phy, tiny_ndop):
    """sigma_3 = 1 and no PHY losses keep PHY at its initial constant c; PO4 and DOP then follow the
    PO4-DOP model with alpha = mu_1 c (same grid and matrices)."""
    c = 0.8
    u = synth.nominal(PHY)
    u[6] = u[7] = u[8] = 0.0      # lambda_3, kappa_3, lambda'_3
    u[9] = 1.0                    # sigma_3: everything produced is grazed
    u2 = synth.nominal(synth.MODEL_NDOP)
    u2[[1, 2, 3, 4, 5, 6]] = u[[1, 2, 3, 4, 5, 10]]
    u2[0] = u[0] * c
    g = tiny_phy.grid
    s, e = g.col_start[7], g.col_start[8]
    rng = np.random.default_rng(22)
    yc = np.vstack([rng.uniform(0.5, 3.0, e - s), rng.uniform(0.0, 0.2, e - s), np.full(e - s, c)])
    q3 = oracle.bgc_column(PHY, 250.0, g.dz[:e - s], yc, u, 2)
    q2 = oracle.bgc_column(synth.MODEL_NDOP, 250.0, g.dz[:e - s], yc[:2], u2, 2)
    assert np.abs(q3[:2] - q2).max() <= 1e-15 * np.abs(q2).max()
    assert np.array_equal(q3[2], np.zeros(e - s))
    y0 = np.column_stack([tiny_phy.initial_state()[:, :2], np.full(tiny_phy.n, c)])
    y3, _ = oracle.Oracle(tiny_phy).year(u, y0)
    y2, _ = oracle.Oracle(tiny_ndop).year(u2, y0[:, :2])
    assert np.abs(y3[:, :2] - y2).max() <= 1e-12 * np.abs(y2).max()
    assert np.abs(y3[:, 2] / c - 1).max() <= 1e-13


def test_phy_linear_losses_closed_form(tiny_phy):
    """Identity transport, mu_1 = kappa_3 = 0: PHY_j = PHY_0 (1 - dt_d (chi lambda_3 + lambda'_3))^j with chi = 1
    in the euphotic zone, and PO4 + DOP + PHY is constant at every point."""
    inp = _identity_transport(tiny_phy)
    u = synth.nominal(PHY)
    u[0] = 0.0
    u[7] = 0.0
    y0 = np.column_stack([np.full(inp.n, 2.0), np.linspace(0.1, 0.5, inp.n), np.linspace(0.05, 0.3, inp.n)])
    y1, _ = oracle.Oracle(inp).year(u, y0)
    dtd = 360.0 / inp.nstep
    g = inp.grid
    layer = np.concatenate([np.arange(g.col_start[c + 1] - g.col_start[c]) for c in range(g.ncol)])
    chi = (layer < inp.neuphotic).astype(float)
    expect = y0[:, 2] * (1 - dtd * (chi * u[6] + u[8])) ** inp.nstep
    assert np.abs(y1[:, 2] / expect - 1).max() < 2e-13
    assert np.abs(y1.sum(1) / y0.sum(1) - 1).max() < 2e-13


def test_phy_quadratic_loss(tiny_phy):
    """Identity transport, mu_1 = lambda_3 = lambda'_3 = 0: euphotic PHY follows PHY <- PHY - dt_d kappa_3 PHY^2,
    within O(dt) of the ODE solution PHY_0 / (1 + kappa_3 PHY_0 t); PHY below is unchanged."""
    inp = _identity_transport(tiny_phy)
    u = synth.nominal(PHY)
    u[0] = u[6] = u[8] = 0.0
    y0 = np.column_stack([np.full(inp.n, 2.0), np.full(inp.n, 0.1), np.linspace(0.05, 0.9, inp.n)])
    y1, _ = oracle.Oracle(inp).year(u, y0)
    dtd = 360.0 / inp.nstep
    g = inp.grid
    layer = np.concatenate([np.arange(g.col_start[c + 1] - g.col_start[c]) for c in range(g.ncol)])
    eu = layer < inp.neuphotic
    p = y0[:, 2].copy()
    for _ in range(inp.nstep):
        p = np.where(eu, p - dtd * u[7] * p * p, p)
    assert np.abs(y1[:, 2] / p - 1).max() < 1e-12
    ode = y0[:, 2] / (1 + u[7] * y0[:, 2] * 360.0)
    assert np.abs(y1[eu, 2] - ode[eu]).max() < 0.05 * ode[eu].max()
    assert np.abs(y1.sum(1) / y0.sum(1) - 1).max() < 2e-13


def test_phy_mass_conserved_and_positive():
    inp = synth.small_ndop(model=PHY)
    u = synth.nominal(PHY)
    y0 = inp.initial_state()
    y1, _ = oracle.Oracle(inp).year(u, y0)
    V = inp.grid.volumes()
    assert abs(V @ y1.sum(1) - V @ y0.sum(1)) <= 1e-13 * (V @ y0.sum(1))
    assert y1.min() > 0.0
    assert np.abs(y1[:, 2] - y0[:, 2]).max() > 1e-3       # PHY changed


def test_phy_derivatives(tiny_phy):
    """Tangent vs central differences, tangent vs reverse (dot test), dJ/du (11 parameters) and dJ/dy0
    vs fourth-order central differences."""
    inp = tiny_phy
    o = oracle.Oracle(inp)
    u = synth.nominal(PHY)
    rng = np.random.default_rng(23)
    y = inp.initial_state() * rng.uniform(0.8, 1.2, size=(inp.n, 3))
    v = rng.standard_normal(y.shape) * y
    w = rng.standard_normal(y.shape)
    _, jv = o.year_tangent(u, y, v)
    h = 1e-5
    fd = (o.year(u, y + h * v)[0] - o.year(u, y - h * v)[0]) / (2 * h)
    assert np.abs(jv - fd).max() < 1e-7 * np.abs(jv).max()
    ybar, _ = o.year_vjp(u, y, w)
    assert np.sum(w * jv) == pytest.approx(np.sum(ybar * v), rel=1e-12)
    obs = _obs(inp)
    y0 = inp.initial_state()
    J, dJdu, dJdy0 = o.year_adjoint(u, y0, obs)
    for p in range(u.size):
        def Jp(x):
            q = u.copy()
            q[p] = x
            return o.year_misfit(q, y0, obs)[0]
        assert dJdu[0, p] == pytest.approx(_fd4(Jp, u[p], 1e-4 * abs(u[p])), rel=1e-6), p
    d = rng.standard_normal(y0.shape) * y0
    fdy = _fd4(lambda s: o.year_misfit(u, y0 + s * d, obs)[0], 0.0, 1e-4)
    assert np.sum(dJdy0 * d) == pytest.approx(fdy, rel=1e-6)
